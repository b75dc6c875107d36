"""Back-propagation through time with the simulator's hand-written adjoint
(Crazyflow, arXiv 2606.01478, Methods, "Backpropagation Through Time"): a policy
is trained on analytical gradients through the unrolled dynamics, with no value
network. The policy is either the linear state feedback of the rollout
objective, u_t = ubar_t + G_w (x_t[0:13] - x_ref(t)), or the small-MLP policy
u_t = ubar_t + W3 tanh(W2 tanh(W1 e_t + b1) + b2) + b3 on the same tracking
error (`policy_hidden` > 0), optionally with the open-loop commands ubar_t as
parameters too; with ``policy_scale`` the output o enters as s * tanh(o), a
normalised action in [-1, 1] mapped onto each command's range. The objective is one of the library's: the tracking loss
(position error to the reference plus w_u |u_t|^2) or, with ``reward`` in
``obj_kw``, minus the paper's BPTT reward (exponential distance term, tilt,
action and action-change penalties). Every rollout and adjoint runs in the HIP
library; Adam is PyTorch's, on the device."""
from __future__ import annotations

from typing import Callable, Dict, Optional

from .binding import RolloutLoss, Sim


def train_policy(sim: Sim, x0, ubar, T: int, params, *, iters: int, lr: float = 4.6e-2,
                 ckpt_every: int = 10, obj_kw: Optional[Dict] = None, dloss=None,
                 train_commands: bool = False, chain: bool = False, reset_every: int = 0,
                 clip_grad_norm: float = 0.0,
                 callback: Optional[Callable[[int, float], None]] = None) -> Dict:
    """Adam on the policy parameters ``params`` (linear gains [G][4][13], or MLP
    policies [G][P] with ``policy_hidden`` in ``obj_kw``) and, with
    ``train_commands``, on ``ubar`` [T][4][D], to lower sum_d dloss_d * loss_d of a
    T-step rollout from ``x0`` [S][D]. Tensors live on the handle's device.
    With ``chain`` each rollout starts from the previous one's final state and
    follows the figure-eight from where the previous one ended (``ref_step0``
    advances by T per iteration), so training covers the whole trajectory;
    ``reset_every`` = n > 0 restarts from ``x0`` (and the first reference step)
    after every n iterations, an episode of n T steps. ``clip_grad_norm`` > 0
    rescales the gradient to at most that norm before each Adam step.
    Returns the per-iteration objective values (a device tensor [iters], read
    once at the end) and the trained parameters."""
    import torch

    params = params.detach().clone().requires_grad_(True)
    ubar = ubar.detach().clone().requires_grad_(train_commands)
    trainable = [params] + ([ubar] if train_commands else [])
    opt = torch.optim.Adam(trainable, lr=lr)
    w = None if dloss is None else dloss.detach()
    losses = torch.empty(iters, dtype=torch.float32, device=params.device)
    kw = dict(obj_kw or {})
    step00 = int(kw.pop("ref_step0", 0))
    step0 = step00
    x = x0
    for it in range(iters):
        opt.zero_grad(set_to_none=True)
        per_drone, x_T = RolloutLoss.apply(x, ubar, params, sim, T, ckpt_every, dict(kw, ref_step0=step0),
                                           return_state=True)
        if chain:
            x = x_T
            step0 += T
            if reset_every and (it + 1) % reset_every == 0:
                x, step0 = x0, step00
        total = per_drone.sum() if w is None else (per_drone * w).sum()
        total.backward()
        if clip_grad_norm > 0:
            torch.nn.utils.clip_grad_norm_(trainable, clip_grad_norm)
        opt.step()
        losses[it] = total.detach()
        if callback is not None:
            callback(it, total)
    return {"gain": params.detach(), "ubar": ubar.detach(), "losses": losses}


def train_linear_policy(sim: Sim, x0, ubar, T: int, gain, **kw) -> Dict:
    """train_policy with the linear feedback gains [G][4][13]."""
    return train_policy(sim, x0, ubar, T, gain, **kw)


def tracking_rms(sim: Sim, x0, ubar, T: int, params, *, ref_amp: float, ref_period: float,
                 policy_hidden: int = 0, ref_offset=None, ref_time_shift=None, policy_scale=None) -> float:
    """Root-mean-square distance of the drones to the reference over a T-step
    rollout under the policy: sqrt(sum_d sum_{t=1..T} |p_t - p_ref(t)|^2 / (D T)),
    the library's tracking loss with no command term."""
    import torch

    obj = Sim.objective(gain=params, ref_amp=ref_amp, ref_period=ref_period, ref_offset=ref_offset, w_u=0.0,
                        policy_hidden=policy_hidden, ref_time_shift=ref_time_shift, policy_scale=policy_scale)
    loss = torch.empty(sim.D, device=x0.device, dtype=torch.float32)
    sim.rollout(x0, ubar, T, obj, T, loss=loss)
    return float((loss.double().sum() / (sim.D * T)).sqrt())
