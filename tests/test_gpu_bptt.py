"""The BPTT tracking setup on the GPU: per-drone reference time shifts (starts
spread along the figure-eight), the reference time offset of chained rollouts,
the squashed (normalised) policy output, each against the oracle's autograd, and
a short training run through the library whose tracking error must fall; Adam
on the feedback gain with the library's rollout and adjoint against the same
Adam driven by the FP64 oracle's autograd gradients."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_helpers import dev
from paper_2606_01478_amd import binding as B
from paper_2606_01478_amd.bptt import tracking_rms, train_linear_policy, train_policy
from test_gpu_mlp import _grads
from test_gpu_parity import _check_against_oracle, _sim

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("hidden", [0, 16])
def test_bptt_setup_paper_scale_against_oracle(gpu_lib, hidden):
    """16 drones, 40 steps at 50 Hz, starts spread over the 10 s figure-eight,
    normalised actions, the paper's reward; the policy trained a little first so
    that it acts (a zero or tiny policy leaves the squash and its VJP untested)."""
    w = W.bptt_tracking(hidden=hidden, out_scale=0.5)
    if not hidden:
        w.gain = W._f32(np.random.Generator(np.random.Philox(70)).normal(0.0, 0.5, size=(1, 4, 13)))
    _check_against_oracle(w, _grads(_sim(w), w, 10))


def test_time_shift_on_tiles_with_offsets_and_linear_policy(gpu_lib):
    """Mixed first-principles (PID) / identified worlds in 64-lane tiles, per-drone
    offsets and random time shifts, the tracking loss (not the reward)."""
    w = W.uneven_mixed_adjoint(seed=71, n_worlds=12, n_subset=8, steps=60, n_max=90)
    rng = np.random.Generator(np.random.Philox(71))
    w.ref_time_shift = W._f32(rng.uniform(-4.0, 8.0, size=w.n_drones_total))
    sim = _sim(w)
    assert sim.launch_config()["tile"] == 64
    _check_against_oracle(w, _grads(sim, w, 15))


def test_reference_time_offset_against_oracle(gpu_lib):
    """Step n tracks the figure-eight at (ref_step0 + n) dt: a rollout that starts
    deep into the reference, with the linear feedback and the tracking loss."""
    w = W.id_rollout_grad(seed=72, n_worlds=100, steps=80)
    w.ref_step0 = 777
    _check_against_oracle(w, _grads(_sim(w), w, 20))


@pytest.mark.parametrize("hidden", [0, 8])
def test_squashed_policy_saturating_against_oracle(gpu_lib, hidden):
    """Policy outputs of order 1-3 (tanh partly saturated) on the identified lane
    kernel, tracking loss, checkpoint every step and every 16 steps."""
    if hidden:
        w = W.id_rollout_grad_mlp(seed=73, n_worlds=90, steps=48, hidden=hidden, out_scale=1.0)
    else:
        w = W.id_rollout_grad(seed=73, n_worlds=90, steps=48, gain_std=2.0)
    w.policy_scale = W._f32([0.4, 0.3, 0.2, 0.1])
    sim = _sim(w)
    _check_against_oracle(w, _grads(sim, w, 16))
    _check_against_oracle(w, _grads(sim, w, 1))


def test_bptt_training_lowers_tracking_error(gpu_lib):
    """The paper's BPTT schedule (16 environments x 40-step rollouts, Adam at
    4.6e-2, 157 iterations) on the small-MLP policy with chained rollouts, episodes
    of 12 rollouts and gradient clipping: the RMS tracking error over 10 s from the
    16 starts must fall from metres to a few centimetres."""
    w = W.bptt_tracking(hidden=16)
    sim = _sim(w)
    x0, ubar, theta0 = dev(w.x0), dev(w.cmds), dev(w.gain)
    shift = dev(w.ref_time_shift)
    ev = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, policy_hidden=16, ref_time_shift=shift,
              policy_scale=w.policy_scale)
    hover = ubar[:1].expand(500, 4, w.n_worlds).contiguous()
    rms0 = tracking_rms(sim, x0, hover, 500, theta0, **ev)
    kw = dict(ev, reward=w.reward, w_u=0.0)
    res = train_policy(sim, x0, ubar, w.steps, theta0, iters=157, lr=4.6e-2, ckpt_every=10, obj_kw=kw,
                       chain=True, reset_every=12, clip_grad_norm=10.0)
    rms1 = tracking_rms(sim, x0, hover, 500, res["gain"], **ev)
    print(f"tracking RMS before {rms0:.4f} m, after {rms1:.4f} m")
    assert sim.last_error() == 0
    assert math.isfinite(rms1) and rms0 > 1.0 and rms1 < 0.1


# ---- Adam through the library vs Adam on the oracle ---------------------------

def _setup(seed=12):
    w = W.small("id_rollout_grad", seed=seed)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    return w, sim, kw


def test_adam_steps_match_oracle_driven_adam(gpu_lib):
    w, sim, kw = _setup()
    lr, iters = 1e-2, 3
    out = train_linear_policy(sim, dev(w.x0), dev(w.cmds), w.steps, dev(w.gain), iters=iters, lr=lr,
                              ckpt_every=10, obj_kw=kw)
    torch.cuda.synchronize()
    b = O.Batch.from_workload(w)
    G = torch.tensor(w.gain, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([G], lr=lr)
    ref_losses, g0 = [], None
    for _ in range(iters):
        opt.zero_grad()
        r = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, gain=G, gain_index=w.gain_index, **kw)
        total = r["loss"].sum()
        total.backward()
        g0 = G.grad.detach().clone() if g0 is None else g0
        opt.step()
        ref_losses.append(float(total.detach()))
    got = out["gain"].double().cpu()
    step_ref = G.detach() - torch.tensor(w.gain, dtype=torch.float64)
    step_got = got - torch.tensor(w.gain, dtype=torch.float64)
    # Adam normalises each coordinate's step, so a coordinate whose gradient is
    # near zero may step either way; where the gradient is significant the
    # device's gradients (within 1e-3) give the same updates to a small
    # fraction of lr
    sig = g0.abs() > 1e-3 * g0.abs().max()
    assert sig.sum() > 10
    err = torch.max(torch.abs(step_got - step_ref)[sig])
    assert err <= 0.05 * lr, err
    gl = out["losses"].double().cpu().numpy()
    assert np.allclose(gl, ref_losses, rtol=1e-4, atol=0)


def test_training_lowers_the_objective(gpu_lib):
    w, sim, kw = _setup(seed=21)
    out = train_linear_policy(sim, dev(w.x0), dev(w.cmds), w.steps, dev(w.gain), iters=40, lr=1e-2,
                              ckpt_every=10, obj_kw=kw, train_commands=True)
    torch.cuda.synchronize()
    losses = out["losses"].cpu().numpy()
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0], (losses[0], losses[-1])
