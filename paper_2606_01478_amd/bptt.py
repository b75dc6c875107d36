"""Back-propagation through time with the simulator's hand-written adjoint
(Crazyflow, arXiv 2606.01478, Methods, "Backpropagation Through Time"): a policy
is trained on analytical gradients through the unrolled dynamics, with no value
network. Here the policy is the linear state feedback of the rollout objective,
u_t = ubar_t + G_w (x_t[0:13] - x_ref(t)), optionally with the open-loop
commands ubar_t as parameters too, and the objective is one of the library's:
the tracking loss (position error to the reference plus w_u |u_t|^2) or, with
``reward`` in ``obj_kw``, minus the paper's BPTT reward (exponential distance
term, tilt, action and action-change penalties). Every rollout and adjoint runs
in the HIP library; Adam is PyTorch's, on the device."""
from __future__ import annotations

from typing import Callable, Dict, Optional

from .binding import RolloutLoss, Sim


def train_linear_policy(sim: Sim, x0, ubar, T: int, gain, *, iters: int, lr: float = 4.6e-2,
                        ckpt_every: int = 10, obj_kw: Optional[Dict] = None, dloss=None,
                        train_commands: bool = False,
                        callback: Optional[Callable[[int, float], None]] = None) -> Dict:
    """Adam on the feedback gains ``gain`` ``[G][4][13]`` (and on ``ubar``
    ``[T][4][D]`` with ``train_commands``) to lower sum_d dloss_d * loss_d of a
    T-step rollout from ``x0`` ``[S][D]``. Tensors live on the handle's device;
    ``gain`` and ``ubar`` are updated in place. Returns the per-iteration
    objective values (a device tensor ``[iters]``, read once at the end) and the
    trained parameters."""
    import torch

    gain = gain.detach().clone().requires_grad_(True)
    ubar = ubar.detach().clone().requires_grad_(train_commands)
    params = [gain] + ([ubar] if train_commands else [])
    opt = torch.optim.Adam(params, lr=lr)
    w = None if dloss is None else dloss.detach()
    losses = torch.empty(iters, dtype=torch.float32, device=gain.device)
    for it in range(iters):
        opt.zero_grad(set_to_none=True)
        per_drone = RolloutLoss.apply(x0, ubar, gain, sim, T, ckpt_every, obj_kw or {})
        total = per_drone.sum() if w is None else (per_drone * w).sum()
        total.backward()
        opt.step()
        losses[it] = total.detach()
        if callback is not None:
            callback(it, total)
    return {"gain": gain.detach(), "ubar": ubar.detach(), "losses": losses}
