"""Parity at the full workload sizes, in the launch configuration bench.py times:
every drone where the oracle finishes in seconds, otherwise drones sampled one
by one (drones never interact) plus properties that hold at any size."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_helpers import assert_grad_close, assert_states_close, dev, sample_drones
from paper_2606_01478_amd import binding as B

pytestmark = pytest.mark.gpu


def test_closed_loop_4096_worlds_all_drones(gpu_lib):
    w = W.fp_pid_closed_loop()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    x = dev(w.x0)
    sim.step_k(x, dev(w.cmds), w.steps)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what="4096 PID worlds x_1000")


def test_swarm_64x4000_chunkings_and_samples(gpu_lib):
    w = W.id_swarm()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    u = dev(w.cmds)
    outs = {}
    for k in (1, 10, 100, 1000):
        x = dev(w.x0)
        for _ in range(w.steps // k):
            sim.step_k(x, u, k)
        outs[k] = x
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(w.n_drones_total, 256, replace=False)
    ws = sample_drones(w, idx)
    ref = O.simulate_held(ws)
    ii = torch.as_tensor(idx, device="cuda")
    for k in (1, 10, 100, 1000):
        assert_states_close(outs[k][:, ii], ref, ws, what=f"64 x 4000 swarm sampled, {k} steps per launch")
        assert_states_close(outs[k], outs[1000], w, what=f"64 x 4000 swarm all drones, {k} vs 1000 steps per launch")


_CONFIG4_ORACLE = {}


def _tracking_oracle(w):
    """The oracle's loss and gradients of the full differentiable workload,
    computed once for the three checkpoint intervals."""
    if "ref" not in _CONFIG4_ORACLE:
        _CONFIG4_ORACLE["ref"] = O.rollout_workload(w, with_grad=True)
    return _CONFIG4_ORACLE["ref"]


@pytest.mark.parametrize("K", [25, 50, 100])
def test_differentiable_1024_worlds(gpu_lib, K):
    w = W.id_rollout_grad()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    T = w.steps
    x0, cmds, gain = dev(w.x0), dev(w.cmds), dev(w.gain)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    ckpt = sim.ckpt_buffer(T, K)
    loss = torch.empty(sim.D, device="cuda")
    sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt, loss=loss)
    g_cmds, g_x0, g_gain = torch.empty_like(cmds), torch.empty_like(x0), torch.empty_like(gain)
    sim.rollout_backward(x0, cmds, T, obj, K, ckpt, dloss=dev(w.dloss), g_cmds=g_cmds, g_x0=g_x0, g_gain=g_gain)
    torch.cuda.synchronize()
    ref = _tracking_oracle(w)
    lr = ref["loss"]
    assert torch.all((loss.double().cpu() - lr).abs() <= 1e-4 * lr.abs().clamp_min(1e-2))
    assert_grad_close(g_cmds, ref["g_cmds"], f"1024 tracking worlds K={K} g_cmds")
    assert_grad_close(g_x0, ref["g_x0"], f"1024 tracking worlds K={K} g_x0")
    assert (g_gain.double().cpu() - ref["g_gain"]).norm() <= 1e-3 * ref["g_gain"].norm()


def test_differentiable_checkpoint_invariance_full(gpu_lib):
    w = W.id_rollout_grad()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    T = w.steps
    x0, cmds, gain = dev(w.x0), dev(w.cmds), dev(w.gain)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    res = {}
    for K in (25, 50, 100):
        ckpt = sim.ckpt_buffer(T, K)
        sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt)
        g = [torch.empty_like(cmds), torch.empty_like(x0), torch.empty_like(gain)]
        sim.rollout_backward(x0, cmds, T, obj, K, ckpt, g_cmds=g[0], g_x0=g[1], g_gain=g[2])
        res[K] = g
    torch.cuda.synchronize()
    # the forward kernel and the adjoint's recompute loop are compiled separately,
    # so states at segment boundaries may differ in the last bit between intervals
    for K in (25, 100):
        for a, b in zip(res[K], res[50]):
            assert ((a - b).abs().max() <= 1e-6 * b.abs().max()).item(), K


def test_uneven_2048_worlds_autotuned_launch(gpu_lib):
    """Full uneven mixed batch (~1M drones) in the autotuned launch configuration,
    512 drones sampled against the oracle. At one chunking (all steps in one
    launch) the per-tile grid, the work queue and the single mixed-model launch
    give the same bits; the autotuned chunking restarts the compensated sums at
    each launch boundary, so it agrees with them to the parity bar."""
    w = W.uneven_mixed()
    sim = B.Sim.from_workload(w)
    x = dev(w.x0)
    u = dev(w.cmds)
    sim.autotune(x, u, w.steps, 1500)
    sim.step_k(x, u, w.steps)
    one = {}
    for name, flags in (("grid", 0), ("wq", B.F_WORKQUEUE), ("single", B.F_SINGLE_LAUNCH)):
        xs = dev(w.x0)
        B.Sim.from_workload(w, flags=flags | B.F_NO_AUTOTUNE_CACHE).step_k(xs, u, w.steps)
        one[name] = xs
    torch.cuda.synchronize()
    assert torch.equal(one["grid"], one["wq"])
    assert torch.equal(one["grid"], one["single"])
    assert_states_close(x, one["grid"], w, what="uneven 2048 worlds autotuned vs one launch")
    idx = np.random.default_rng(1).choice(w.n_drones_total, 512, replace=False)
    ws = sample_drones(w, idx)
    assert_states_close(x[:, torch.as_tensor(idx, device="cuda")], O.simulate_held(ws), ws, what="uneven 2048 worlds sampled")


def test_uneven_adjoint_subset_full(gpu_lib):
    """256-world subset, T = 1000: per-drone gradients on sampled drones vs the
    oracle; the gain gradient against sum_t sum_d g_cmds[t] e_t^T computed from
    the full trajectory (an identity that holds at any size)."""
    w = W.uneven_mixed_adjoint()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    T, K = w.steps, 50
    x0, cmds, gain, off = dev(w.x0), dev(w.cmds), dev(w.gain), dev(w.ref_offset)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, ref_offset=off, w_u=w.w_u)
    ckpt = sim.ckpt_buffer(T, K)
    traj = torch.empty((T + 1, sim.S, sim.D), device="cuda")
    loss = torch.empty(sim.D, device="cuda")
    sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt, traj=traj, loss=loss)
    g_cmds, g_x0, g_gain = torch.empty_like(cmds), torch.empty_like(x0), torch.empty_like(gain)
    sim.rollout_backward(x0, cmds, T, obj, K, ckpt, dloss=dev(w.dloss), g_cmds=g_cmds, g_x0=g_x0, g_gain=g_gain)
    torch.cuda.synchronize()
    # sampled drones vs the oracle
    idx = np.random.default_rng(2).choice(w.n_drones_total, 48, replace=False)
    ws = sample_drones(w, idx)
    ref = O.rollout_workload(ws, with_grad=True)
    ii = torch.as_tensor(idx, device="cuda")
    lr = ref["loss"]
    assert torch.all((loss[ii].double().cpu() - lr).abs() <= 1e-4 * lr.abs().clamp_min(1e-2))
    assert_grad_close(g_cmds[:, :, ii], ref["g_cmds"], "uneven subset g_cmds")
    gx, rx = g_x0[:, ii].double().cpu(), ref["g_x0"].clone()
    idm = torch.as_tensor(ws.model_per_world == W.MODEL_ID)
    gx[13:, idm] = 0
    rx[13:, idm] = 0
    assert_grad_close(gx, rx, "uneven subset g_x0")
    # gain gradient identity on the full subset
    world = np.repeat(np.arange(w.n_worlds), w.drones_per_world)
    models = torch.as_tensor(w.model_per_world[world], device="cuda")
    D = w.n_drones_total
    t = torch.arange(T, device="cuda", dtype=torch.float64) * np.float32(w.dt)
    w0 = 2 * np.pi / w.ref_period
    xr = torch.zeros((T, 13, D), device="cuda", dtype=torch.float64)
    xr[:, 0] = (w.ref_amp * torch.sin(w0 * t))[:, None]
    xr[:, 1] = (0.5 * w.ref_amp * torch.sin(2 * w0 * t))[:, None]
    xr[:, 0:3] += off.double()[None]
    vx = (w.ref_amp * w0 * torch.cos(w0 * t))[:, None]
    vy = (w.ref_amp * w0 * torch.cos(2 * w0 * t))[:, None]
    fp = models == W.MODEL_FP
    xr[:, 6] = torch.where(fp, 1.0, 0.0)
    xr[:, 7] = torch.where(fp, vx, 0.0)
    xr[:, 8] = torch.where(fp, vy, 0.0)
    xr[:, 6] = torch.where(fp, xr[:, 6], vx)
    xr[:, 7] = torch.where(fp, xr[:, 7], vy)
    mg = torch.as_tensor(w.params["mass"][world, 0] * w.params["gravity"][world, 0] / np.where(
        w.params["c_f"][world, 0] > 0, w.params["c_f"][world, 0], 1.0), device="cuda", dtype=torch.float64)
    xr[:, 12] = torch.where(fp, xr[:, 12], mg[None])
    e = traj[:T, 0:13].double() - xr
    gidx = torch.as_tensor(w.gain_index[world], device="cuda")
    for k in range(gain.shape[0]):
        sel = gidx == k
        gk = g_cmds[:, :, sel].double().permute(1, 0, 2).reshape(4, -1)
        ek = e[:, :, sel].permute(1, 0, 2).reshape(13, -1).t().contiguous()
        expect = gk @ ek
        assert (g_gain[k].double() - expect).norm() <= 1e-3 * expect.norm(), k


def test_goal_gradient_2p20_worlds_sampled(gpu_lib):
    """The gradient-throughput workload at full size (2^20 single-drone worlds,
    10 steps, one checkpoint): per-drone loss and gradients of 256 sampled drones
    vs the oracle; the per-drone results do not depend on the batch."""
    w = W.gradient_goal()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    T = w.steps
    x0, cmds, off = dev(w.x0), dev(w.cmds), dev(w.ref_offset)
    obj = B.Sim.objective(ref_amp=w.ref_amp, ref_period=w.ref_period, ref_offset=off, w_u=w.w_u)
    ckpt = sim.ckpt_buffer(T, T)
    loss = torch.empty(sim.D, device="cuda")
    sim.rollout(x0, cmds, T, obj, T, ckpt=ckpt, loss=loss)
    g_cmds, g_x0 = torch.empty_like(cmds), torch.empty_like(x0)
    sim.rollout_backward(x0, cmds, T, obj, T, ckpt, dloss=dev(w.dloss), g_cmds=g_cmds, g_x0=g_x0)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(3).choice(w.n_drones_total, 256, replace=False))
    ws = W.subset(w, idx)
    ref = O.rollout_workload(ws, with_grad=True)
    ii = torch.as_tensor(idx, device="cuda")
    lr = ref["loss"]
    assert torch.all((loss[ii].double().cpu() - lr).abs() <= 1e-4 * lr.abs().clamp_min(1e-2))
    assert_grad_close(g_cmds[:, :, ii], ref["g_cmds"], "goal g_cmds")
    assert_grad_close(g_x0[:, ii], ref["g_x0"], "goal g_x0")


def _interface_case(name):
    n, T = 1 << 20, 100
    if name == "torque":
        return W.fp_torque(n_worlds=n, steps=T)
    if name == "position":
        return W.fp_position(n_worlds=n, steps=T)
    return dataclasses.replace(W.fp_pid_closed_loop(n_worlds=n, steps=T), ctrl_every=5)


@pytest.mark.parametrize("name", ["torque", "position", "pid_every_5"])
def test_interfaces_2p20_worlds_sampled(gpu_lib, name):
    """The interface measurement's workloads (2^20 single-drone worlds, 100 held
    steps, launch shape autotuned as the measurement does): 256 sampled drones
    against the oracle, and every state finite."""
    w = _interface_case(name)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    x, u = dev(w.x0), dev(w.cmds)
    sim.autotune(x, u, w.steps, 300)
    sim.step_k(x, u, w.steps)
    torch.cuda.synchronize()
    assert sim.last_error() == 0
    assert bool(torch.isfinite(x).all())
    idx = np.random.default_rng(7).choice(w.n_drones_total, 256, replace=False)
    ws = sample_drones(w, idx)
    ii = torch.as_tensor(idx, device="cuda")
    assert_states_close(x[:, ii], O.simulate_held(ws), ws, what=f"{name} 2^20 worlds, sampled")
    sim.close()


def test_shared_gain_gradient_over_2p20_worlds(gpu_lib):
    """2^20 single-drone identified worlds sharing one 4x13 gain, 10 steps: the
    gain gradient (a fixed-order two-stage reduction over the drones) is
    bit-identical across calls and equals sum_t sum_d g_cmds[t, :, d] e_t[d]^T
    evaluated in float64 from the trajectory."""
    w = W.id_rollout_grad(seed=95, n_worlds=1 << 20, steps=10)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    T, D = w.steps, w.n_drones_total
    x0, cmds, gain = dev(w.x0), dev(w.cmds), dev(w.gain)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    ckpt = sim.ckpt_buffer(T, T)
    traj = torch.empty((T + 1, sim.S, D), device="cuda")
    sim.rollout(x0, cmds, T, obj, T, ckpt=ckpt, traj=traj)
    g_cmds = torch.empty_like(cmds)
    gg = [torch.empty_like(gain), torch.empty_like(gain)]
    for g in gg:
        sim.rollout_backward(x0, cmds, T, obj, T, ckpt, g_cmds=g_cmds, g_gain=g)
    torch.cuda.synchronize()
    assert torch.equal(gg[0], gg[1])
    t = torch.arange(T, device="cuda", dtype=torch.float64) * np.float32(w.dt)
    w0 = 2 * np.pi / w.ref_period
    xr = torch.zeros((T, 13, 1), device="cuda", dtype=torch.float64)
    xr[:, 0, 0] = w.ref_amp * torch.sin(w0 * t)
    xr[:, 1, 0] = 0.5 * w.ref_amp * torch.sin(2 * w0 * t)
    xr[:, 6, 0] = w.ref_amp * w0 * torch.cos(w0 * t)
    xr[:, 7, 0] = w.ref_amp * w0 * torch.cos(2 * w0 * t)
    xr[:, 12, 0] = float(np.float32(W.MASS) * np.float32(W.GRAVITY) / np.float32(W.ID_CF))
    ref = torch.zeros((4, 13), device="cuda", dtype=torch.float64)
    for n in range(T):
        e = traj[n, 0:13].double() - xr[n]
        ref += g_cmds[n].double() @ e.T
    err = (gg[0][0].double() - ref).norm() / ref.norm()
    assert err <= 1e-4, err
