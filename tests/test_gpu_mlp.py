"""The small-MLP policy (BPTT actor) in the rollout and its hand-written VJP
against the oracle's autograd: loss, final state and gradients with respect to
the per-step commands, the initial state and every policy parameter."""
import ctypes
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_helpers import assert_grad_close, dev
from paper_2606_01478_amd import binding as B
from test_gpu_parity import _check_against_oracle, _rollout_grads, _sim

pytestmark = pytest.mark.gpu


def _mlp(w, hidden, seed, out_scale=0.02):
    rng = np.random.Generator(np.random.Philox(seed))
    n_pol = 1 if w.gain is None else w.gain.shape[0]
    return dataclasses.replace(w, gain=W.mlp_policy_params(rng, n_pol, hidden, out_scale), policy_hidden=hidden)


def _obj(w):
    return B.Sim.objective(gain=dev(w.gain), ref_amp=w.ref_amp, ref_period=w.ref_period,
                           ref_offset=None if w.ref_offset is None else dev(w.ref_offset), w_u=w.w_u,
                           reward=w.reward, policy_hidden=w.policy_hidden, ref_step0=w.ref_step0,
                           ref_time_shift=None if w.ref_time_shift is None else dev(w.ref_time_shift),
                           policy_scale=w.policy_scale)


def _grads(sim, w, K, noalloc=False):
    T = w.steps
    x0, cmds = dev(w.x0), dev(w.cmds)
    obj = _obj(w)
    ckpt = sim.ckpt_buffer(T, K, int(obj.kind))
    loss = torch.empty(sim.D, device="cuda")
    lw = torch.empty(sim.n_worlds, device="cuda")
    xT = torch.empty_like(x0)
    sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt, x_T=xT, loss=loss, loss_world=lw)
    g = dict(g_cmds=torch.empty_like(cmds), g_x0=torch.empty_like(x0), g_gain=torch.empty_like(dev(w.gain)))
    back = sim.rollout_backward_noalloc if noalloc else sim.rollout_backward
    back(x0, cmds, T, obj, K, ckpt, dloss=dev(w.dloss), **g)
    torch.cuda.synchronize()
    return dict(loss=loss, loss_world=lw, x=xT, **g)


@pytest.mark.parametrize("hidden", [8, 32])
def test_mlp_identified_lane_kernel(gpu_lib, hidden):
    """100 single-drone identified worlds (one drone per lane), 80 steps, one policy."""
    w = W.id_rollout_grad_mlp(seed=60, n_worlds=100, steps=80, hidden=hidden)
    _check_against_oracle(w, _grads(_sim(w), w, 20))


def test_mlp_mixed_tiles_two_policies_reward(gpu_lib):
    """First-principles (PID) and identified worlds in 64-lane tiles, a policy per
    model (width 16), the paper's BPTT reward, checkpoint every 10 steps."""
    w = _mlp(W.uneven_mixed_adjoint(seed=61, n_worlds=12, n_subset=8, steps=60, n_max=140), 16, 61)
    w.reward = W.BPTT_REWARD
    sim = _sim(w)
    assert sim.launch_config()["tile"] == 64
    _check_against_oracle(w, _grads(sim, w, 10))


def test_mlp_slow_controller(gpu_lib):
    """The PID every third step with the policy in front of it (width 8)."""
    w = _mlp(W.uneven_mixed_adjoint(seed=62, n_worlds=10, n_subset=6, steps=61, n_max=50), 8, 62)
    w.ctrl_every = 3
    _check_against_oracle(w, _grads(_sim(w, ctrl_every=3), w, 3))


def test_mlp_checkpoint_interval_invariance_and_noalloc(gpu_lib):
    w = W.id_rollout_grad_mlp(seed=63, n_worlds=70, steps=60, hidden=16)
    sim = _sim(w)
    base = _grads(sim, w, 60)
    for K in (1, 7):
        g = _grads(sim, w, K)
        for k in ("loss", "g_cmds", "g_x0", "g_gain"):
            a, b = g[k], base[k]
            assert ((a - b).abs().max() <= 1e-5 * b.abs().max()).item(), (K, k)
    na = _grads(sim, w, 7, noalloc=True)
    for k in ("g_cmds", "g_x0", "g_gain"):
        assert torch.equal(na[k], _grads(sim, w, 7)[k]), k


def test_mlp_through_rollout_loss(gpu_lib):
    w = W.id_rollout_grad_mlp(seed=64, n_worlds=40, steps=50, hidden=16)
    sim = _sim(w)
    x0 = dev(w.x0).requires_grad_(True)
    cmds = dev(w.cmds).requires_grad_(True)
    theta = dev(w.gain).requires_grad_(True)
    loss = B.RolloutLoss.apply(x0, cmds, theta, sim, w.steps, 10,
                               dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u,
                                    policy_hidden=w.policy_hidden))
    (loss * dev(w.dloss)).sum().backward()
    ref = O.rollout_workload(w, with_grad=True)
    assert_grad_close(cmds.grad, ref["g_cmds"], "mlp g_cmds")
    assert_grad_close(x0.grad, ref["g_x0"], "mlp g_x0")
    assert (theta.grad.double().cpu() - ref["g_gain"]).norm() <= 1e-3 * ref["g_gain"].norm()


def test_mlp_argument_checks(gpu_lib):
    w = W.id_rollout_grad_mlp(seed=65, n_worlds=20, steps=10, hidden=8)
    sim = _sim(w)
    x0, cmds = dev(w.x0), dev(w.cmds)
    bad = B.Sim.objective(gain=dev(w.gain), policy_hidden=33)
    st = sim._lib.cf_rollout(sim._h, x0.data_ptr(), cmds.data_ptr(), 10, ctypes.byref(bad), 10, None, None, None,
                             None, None)
    assert st == B.CF_EINVAL
    # six width-32 policies and the activations do not fit the 64 KiB of LDS
    w6 = W.id_rollout_grad(seed=66, n_worlds=12, steps=10)
    w6.gain_index = np.arange(12, dtype=np.int32) % 6
    w6 = _mlp(dataclasses.replace(w6, gain=np.zeros((6, 4, 13), np.float32)), 32, 66)
    sim6 = _sim(w6)
    obj6 = _obj(w6)
    st = sim6._lib.cf_rollout(sim6._h, dev(w6.x0).data_ptr(), dev(w6.cmds).data_ptr(), 10, ctypes.byref(obj6), 10,
                              None, None, None, None, None)
    assert st == B.CF_EUNSUPPORTED
