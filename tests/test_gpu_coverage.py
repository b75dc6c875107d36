"""GPU parity cases that close gaps in the coverage of the method's options:
the plain kernel against the unrounded oracle, the checkpoint interval the
benchmark times (K = 1) on the mixed batch with the tracking loss, explicit
Euler in the adjoint, the rotor law with distinct acceleration/deceleration
coefficients and a quadratic term, and the checkpoint-buffer contract (several
forwards before their backwards, buffers overwritten in between)."""
import ctypes
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_helpers import assert_grad_close, assert_states_close, dev, sample_drones
from paper_2606_01478_amd import binding as B
from test_gpu_parity import _check_against_oracle, _rollout_grads, _sim

pytestmark = pytest.mark.gpu

EULER, RK4 = W.INTEG_EULER, W.INTEG_RK4


# ---- the plain single-step kernel against the unrounded oracle -----------------------

def test_plain_kernel_closed_loop_against_unrounded_oracle(gpu_lib):
    """One launch per step for 1000 steps of the PID closed loop (200 worlds),
    compared with the oracle that keeps its state in FP64 throughout."""
    w = W.small("fp_pid_closed_loop", seed=2)
    sim = _sim(w, flags=B.F_PLAIN_KERNEL)
    x = dev(w.x0)
    sim.step_k(x, dev(w.cmds), w.steps)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what="plain kernel vs unrounded oracle")


# ---- the timed adjoint configuration -----------------------------------------------------

def test_mixed_subset_tracking_adjoint_checkpoint_every_step(gpu_lib):
    """The 256-world subset of the uneven batch (first-principles PID and
    identified worlds, one launch per model on two streams), T = 1000, the
    tracking loss with feedback, a checkpoint at every step (K = 1, the interval
    the benchmark tunes to): 48 sampled drones against the oracle's autograd and
    every drone against K = 50."""
    w = W.uneven_mixed_adjoint()
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    assert sim.launch_config()["per_model_launches"] == 1
    T = w.steps
    x0, cmds, gain, off = dev(w.x0), dev(w.cmds), dev(w.gain), dev(w.ref_offset)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, ref_offset=off, w_u=w.w_u)
    res = {}
    for K in (1, 50):
        ckpt = sim.ckpt_buffer(T, K)
        loss = torch.empty(sim.D, device="cuda")
        sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt, loss=loss)
        g = (torch.empty_like(cmds), torch.empty_like(x0), torch.empty_like(gain))
        sim.rollout_backward(x0, cmds, T, obj, K, ckpt, dloss=dev(w.dloss), g_cmds=g[0], g_x0=g[1], g_gain=g[2])
        torch.cuda.synchronize()
        res[K] = (loss,) + g
        del ckpt
    idx = np.random.default_rng(5).choice(w.n_drones_total, 48, replace=False)
    ws = sample_drones(w, idx)
    ref = O.rollout_workload(ws, with_grad=True)
    ii = torch.as_tensor(idx, device="cuda")
    loss, g_cmds, g_x0, _ = res[1]
    lr = ref["loss"]
    assert torch.all((loss[ii].double().cpu() - lr).abs() <= 1e-4 * lr.abs().clamp_min(1e-2))
    assert_grad_close(g_cmds[:, :, ii], ref["g_cmds"], "subset K=1 g_cmds")
    gx, rx = g_x0[:, ii].double().cpu(), ref["g_x0"].clone()
    idm = torch.as_tensor(ws.model_per_world == W.MODEL_ID)
    gx[13:, idm] = 0
    rx[13:, idm] = 0
    assert_grad_close(gx, rx, "subset K=1 g_x0")
    # every drone: K = 1 recomputes each step from a binary32 checkpoint, K = 50
    # from registers; both linearise the same discrete map
    idm_all = torch.as_tensor(w.model_per_world[np.repeat(np.arange(w.n_worlds), w.drones_per_world)]
                              == W.MODEL_ID, device="cuda")
    assert (res[1][2][13:, idm_all] == 0).all()   # rows identified drones do not use
    for a, b, name in zip(res[1], res[50], ("loss", "g_cmds", "g_x0", "g_gain")):
        assert ((a - b).abs().max() <= 1e-4 * b.abs().max()).item(), name


# ---- explicit Euler through the adjoint ----------------------------------------------

def _euler(w):
    return dataclasses.replace(w, integrator=EULER)


def test_euler_rotor_interface_rollout_gradients(gpu_lib):
    w = _euler(W.fp_rotor_open_loop(seed=80, n_worlds=70, steps=60))
    w.ref_offset = w.x0[0:3].copy()
    w.dloss = np.linspace(0.5, 1.5, 70).astype(np.float32)
    w.w_u = 1e-9
    _check_against_oracle(w, _rollout_grads(w, 16))


def test_euler_mixed_pid_and_identified_rollout_gradients(gpu_lib):
    """First-principles worlds behind the attitude PID and identified worlds,
    Euler, feedback, per-drone offsets, one gain per model."""
    w = _euler(W.uneven_mixed_adjoint(seed=81, n_worlds=12, n_subset=8, steps=120, n_max=70))
    _check_against_oracle(w, _rollout_grads(w, 40))


def test_euler_identified_rollout_gradients(gpu_lib):
    w = _euler(W.small("id_rollout_grad", seed=82))
    _check_against_oracle(w, _rollout_grads(w, 25))


@pytest.mark.parametrize("k_launch", [1, 100])
def test_euler_identified_held_steps(gpu_lib, k_launch):
    """Identified swarm worlds (tiles with a ragged tail), 1000 Euler steps."""
    w = _euler(W.small("id_swarm", seed=83))
    sim = _sim(w)
    x, u = dev(w.x0), dev(w.cmds)
    for _ in range(w.steps // k_launch):
        sim.step_k(x, u, k_launch)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what=f"identified Euler, {k_launch} steps per launch")


@pytest.mark.parametrize("wq", [False, True])
def test_euler_mixed_held_steps(gpu_lib, wq):
    """First-principles worlds behind the attitude PID and identified worlds, uneven
    sizes, 300 Euler held steps (grid tiles and the work queue)."""
    w = _euler(W.small("uneven_mixed", seed=85))
    sim = _sim(w, flags=B.F_WORKQUEUE if wq else 0)
    x = dev(w.x0)
    sim.step_k(x, dev(w.cmds), w.steps)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what="mixed Euler held steps")


# ---- rotor law with distinct acceleration / deceleration coefficients -------------------

# c_v and c_d when the command is at least the speed (accelerating) and otherwise;
# the quadratic terms add about 15 and 30 1/s to the linear rates near hover
MOTOR_UP = (1.0 / 0.025, 5e-4)
MOTOR_DOWN = (1.0 / 0.05, 1e-3)


def _asymmetric(w):
    fp = w.model_per_world == W.MODEL_FP
    w.params["motor_up"][fp] = MOTOR_UP
    w.params["motor_down"][fp] = MOTOR_DOWN
    return w


def _branch_switches(w, steps):
    """How often, from one step to the next, a rotor of the rotor interface goes
    from accelerating (command at least its speed) to decelerating or back, in
    the oracle's run."""
    b = O.Batch.from_workload(w)
    x = O.t64(w.x0)
    n = 0
    prev = None
    with torch.no_grad():
        for t in range(steps):
            u = O.t64(w.cmds[t] if w.cmds.ndim == 3 else w.cmds)
            up = u >= x[13:17]
            if prev is not None:
                n += int((up != prev).sum())
            prev = up
            x = b.step(x, u)
    return n


@pytest.mark.parametrize("integ", [RK4, EULER])
def test_asymmetric_rotor_law_open_loop(gpu_lib, integ):
    """Per-step rotor commands around hover (every rotor's command crosses its
    speed many times), 500 steps, trajectory and x_T."""
    w = _asymmetric(W.fp_rotor_open_loop(seed=84, integrator=integ))
    assert _branch_switches(w, 100) > 100
    sim = _sim(w)
    T = w.steps
    x0, cmds = dev(w.x0), dev(w.cmds)
    xT = torch.empty_like(x0)
    traj = torch.empty((T + 1, sim.S, sim.D), device="cuda")
    sim.rollout(x0, cmds, T, None, 50, x_T=xT, traj=traj)
    torch.cuda.synchronize()
    with torch.no_grad():
        ref = O.rollout(O.Batch.from_workload(w), O.t64(w.x0), O.t64(w.cmds), T, with_loss=False, keep_traj=True)
    assert_states_close(xT, ref["x"], w, what="asymmetric rotors x_T")
    for t in (1, 10, 100, 250):
        assert_states_close(traj[t], ref["traj"][t], w, what=f"asymmetric rotors traj[{t}]")


@pytest.mark.parametrize("wq", [False, True])
def test_asymmetric_rotor_law_closed_loop(gpu_lib, wq):
    """The attitude PID moves every rotor command up and down through the run:
    1000 held-command steps of 200 worlds, fused or work-queue launch."""
    w = _asymmetric(W.small("fp_pid_closed_loop", seed=85))
    sim = _sim(w, flags=B.F_WORKQUEUE if wq else 0)
    x = dev(w.x0)
    sim.step_k(x, dev(w.cmds), w.steps)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what="asymmetric rotors, PID closed loop")


def test_asymmetric_rotor_law_rollout_gradients_rotor_interface(gpu_lib):
    w = _asymmetric(W.fp_rotor_open_loop(seed=86, n_worlds=70, steps=60))
    w.ref_offset = w.x0[0:3].copy()
    w.dloss = np.linspace(0.5, 1.5, 70).astype(np.float32)
    w.w_u = 1e-9
    _check_against_oracle(w, _rollout_grads(w, 16))


def test_asymmetric_rotor_law_rollout_gradients_mixed(gpu_lib):
    w = _asymmetric(W.uneven_mixed_adjoint(seed=87, n_worlds=12, n_subset=8, steps=120, n_max=70))
    _check_against_oracle(w, _rollout_grads(w, 40))


# ---- the checkpoint-buffer contract ----------------------------------------------------

def test_two_forwards_before_their_backwards(gpu_lib):
    """Two forwards into two buffers, then their backwards in reverse order:
    each backward gives what it gives right after its own forward."""
    w = W.small("id_rollout_grad", seed=90)
    sim = _sim(w)
    T, K = w.steps, 25
    x0, gain = dev(w.x0), dev(w.gain)
    cm = [dev(w.cmds), (dev(w.cmds) * 1.01).contiguous()]
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)

    def grads(c, ck):
        g = torch.empty_like(c)
        sim.rollout_backward(x0, c, T, obj, K, ck, g_cmds=g)
        return g

    ref = []
    for c in cm:
        ck = sim.ckpt_buffer(T, K)
        sim.rollout(x0, c, T, obj, K, ckpt=ck)
        ref.append(grads(c, ck))
    cks = [sim.ckpt_buffer(T, K), sim.ckpt_buffer(T, K)]
    for c, ck in zip(cm, cks):
        sim.rollout(x0, c, T, obj, K, ckpt=ck)
    got = [grads(cm[1], cks[1]), grads(cm[0], cks[0])][::-1]
    torch.cuda.synchronize()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    assert not torch.equal(ref[0], ref[1])
    assert sim.last_error() == 0


@pytest.mark.parametrize("reward", [False, True])
def test_sum_of_two_rollout_losses_backward(gpu_lib, reward):
    """loss(ubar) + loss(1.01 ubar) through RolloutLoss on one handle, one
    backward: the gradient is g(ubar) + 1.01 g(1.01 ubar) of the oracle."""
    w = W.small("id_rollout_grad", seed=91)
    if reward:
        w.reward = W.BPTT_REWARD
    sim = _sim(w)
    x0 = dev(w.x0).requires_grad_(True)
    cmds = dev(w.cmds).requires_grad_(True)
    gain = dev(w.gain).requires_grad_(True)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u, reward=w.reward)
    l1 = B.RolloutLoss.apply(x0, cmds, gain, sim, w.steps, 25, kw)
    l2 = B.RolloutLoss.apply(x0, cmds * 1.01, gain, sim, w.steps, 10, kw)
    (l1.sum() + l2.sum()).backward()
    torch.cuda.synchronize()
    w2 = dataclasses.replace(w, cmds=(w.cmds.astype(np.float32) * np.float32(1.01)).astype(np.float32))
    r1 = O.rollout_workload(w, with_grad=True)
    r2 = O.rollout_workload(w2, with_grad=True)
    assert_grad_close(cmds.grad, r1["g_cmds"] + 1.01 * r2["g_cmds"], "sum of two losses: g_cmds")
    assert_grad_close(x0.grad, r1["g_x0"] + r2["g_x0"], "sum of two losses: g_x0")
    rg = r1["g_gain"] + r2["g_gain"]
    assert (gain.grad.double().cpu() - rg).norm() <= 1e-3 * rg.norm()


def test_backward_after_the_buffer_was_overwritten(gpu_lib):
    """A buffer filled by this handle's forward and then by another handle's
    forward of the same shape: the backward finds the other tag on the device,
    writes NaN gradients and the handle reports CF_ESTATE."""
    w = W.small("id_rollout_grad", seed=92)
    a, b = _sim(w), _sim(w)
    T, K = w.steps, 25
    x0, cmds, gain = dev(w.x0), dev(w.cmds), dev(w.gain)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    ck = a.ckpt_buffer(T, K)
    a.rollout(x0, cmds, T, obj, K, ckpt=ck)
    b.rollout(x0, cmds, T, obj, K, ckpt=ck)
    g = torch.zeros_like(cmds)
    gg = torch.zeros_like(gain)
    a.rollout_backward(x0, cmds, T, obj, K, ck, g_cmds=g, g_gain=gg)
    torch.cuda.synchronize()
    assert torch.isnan(g).all() and torch.isnan(gg).all()
    assert a.last_error() == B.CF_ESTATE
    assert b.last_error() == 0
    # the other handle's own backward of that buffer is fine
    g2 = torch.empty_like(cmds)
    b.rollout_backward(x0, cmds, T, obj, K, ck, g_cmds=g2)
    torch.cuda.synchronize()
    assert torch.isfinite(g2).all() and b.last_error() == 0


def test_backward_refuses_a_different_objective(gpu_lib):
    w = W.small("id_rollout_grad", seed=93)
    sim = _sim(w)
    T, K = w.steps, 25
    x0, cmds, gain = dev(w.x0), dev(w.cmds), dev(w.gain)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    ck = sim.ckpt_buffer(T, K)
    sim.rollout(x0, cmds, T, obj, K, ckpt=ck)
    g = torch.empty_like(cmds)
    for other in (B.Sim.objective(gain=None, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u),
                  B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=2 * w.w_u),
                  B.Sim.objective(gain=gain, ref_amp=0.5, ref_period=w.ref_period, w_u=w.w_u)):
        st = sim._lib.cf_rollout_backward(sim._h, x0.data_ptr(), cmds.data_ptr(), T, ctypes.byref(other), K,
                                          ck.data_ptr(), None, g.data_ptr(), None, None)
        assert st == B.CF_ESTATE
    sim.rollout_backward(x0, cmds, T, obj, K, ck, g_cmds=g)
    torch.cuda.synchronize()
    assert torch.isfinite(g).all() and sim.last_error() == 0


# ---- per-launch timing --------------------------------------------------------------

@pytest.mark.parametrize("graph", [False, True])
def test_launch_times_of_a_mixed_handle(gpu_lib, graph):
    """CF_F_TIMING: one duration per kernel launch of the latest cf_step_k, on
    the stream of each model; the launches fit inside the call's wall time and
    the states equal those of an untimed handle."""
    w = W.small("uneven_mixed", seed=94)
    flags = B.F_WORKQUEUE | B.F_TIMING | (B.F_GRAPH if graph else 0)
    sim = _sim(w, flags=flags)
    ref = _sim(w, flags=B.F_WORKQUEUE)
    x, xr, u = dev(w.x0), dev(w.x0), dev(w.cmds)
    for _ in range(3):   # the graph is captured at the first call and replayed after
        sim.step_k(x, u, 300)
        ref.step_k(xr, u, 300)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    sim.step_k(x, u, 300)
    b.record()
    ref.step_k(xr, u, 300)
    torch.cuda.synchronize()
    total = a.elapsed_time(b)
    assert torch.equal(x, xr)
    cfg = sim.launch_config()
    n_launch = 1 if cfg["chunk"] <= 0 else -(-300 // cfg["chunk"])
    t0, t1 = sim.launch_times(0), sim.launch_times(1)
    if graph:   # the replay is timed as a whole
        assert len(t0) == 1 and len(t1) == 0, (t0, t1)
    else:
        assert len(t0) == n_launch and len(t1) == n_launch, (t0, t1)
    for t in t0 + t1:
        assert 0.0 < t <= total * 1.05 + 0.05
    assert sum(t0) <= total * 1.05 + 0.05
    with pytest.raises(B.CfError):
        ref.launch_times(0)


@pytest.mark.parametrize("cap", [2, 4, 8])
def test_work_queue_wave_cap_gives_identical_states(gpu_lib, cap):
    """Capping the work queue's resident waves per compute unit changes only
    which workgroup takes which tile: the states are bit-identical."""
    w = W.small("uneven_mixed", seed=99)
    a, b = _sim(w, flags=B.F_WORKQUEUE), _sim(w, flags=B.F_WORKQUEUE)
    cfg = a.launch_config()
    b.set_launch_config(1, cfg["tile"], cfg["chunk"], cfg["per_model_launches"], cap)
    xa, xb, u = dev(w.x0), dev(w.x0), dev(w.cmds)
    a.step_k(xa, u, 200)
    b.step_k(xb, u, 200)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    with pytest.raises(B.CfError):
        b.set_launch_config(1, 64, 0, 1, 129)
