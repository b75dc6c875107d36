"""Onboard controller slower than the physics (cf_desc.ctrl_every = n > 1): the
attitude PID, position controller and torque allocation run at the start of
every block of n physics steps with period n dt, their rotor commands held over
the block. GPU vs the FP64 oracle through the C ABI: held steps (fused, work
queue, plain), rollouts and their adjoint with checkpoint intervals shorter
than, equal to and longer than the block, the sampled-rollout controller, and
the argument checks."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_helpers import assert_states_close, dev
from oracle import mppi as OM
from paper_2606_01478_amd import binding as B
from test_gpu_parity import _check_against_oracle, _rollout_grads, _torque_rollout_workload

pytestmark = pytest.mark.gpu


def _sim(w, flags=0):
    return B.Sim.from_workload(w, flags=flags | B.F_NO_AUTOTUNE_CACHE)


@pytest.mark.parametrize("mode", ["grid", "wq", "plain"])
def test_pid_every_fifth_step_held(gpu_lib, mode):
    """Attitude PID every 5 physics steps, 200 single-drone worlds, 1000 steps;
    the plain kernel launches once per block and stores the binary32 state, so
    its reference rounds the state after every block."""
    w = W.small("fp_pid_closed_loop", seed=2)
    w.ctrl_every = 5
    flags = {"grid": 0, "wq": B.F_WORKQUEUE, "plain": B.F_PLAIN_KERNEL}[mode]
    sim = _sim(w, flags)
    x = dev(w.x0)
    sim.step_k(x, dev(w.cmds), w.steps)
    torch.cuda.synchronize()
    ref = O.simulate_held(w, store_every=5 if mode == "plain" else None)
    assert_states_close(x, ref, w, what=f"pid every 5 ({mode})")


def test_pid_every_fifth_step_in_chunks(gpu_lib):
    """The same run as 20 calls of 50 steps: blocks restart with every call."""
    w = W.small("fp_pid_closed_loop", seed=2)
    w.ctrl_every = 5
    sim = _sim(w)
    x, u = dev(w.x0), dev(w.cmds)
    for _ in range(20):
        sim.step_k(x, u, 50)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what="pid every 5, 20 calls")


@pytest.mark.parametrize("control", [W.CTRL_TORQUE, W.CTRL_POSITION])
def test_torque_and_position_interfaces_slow_controller(gpu_lib, control):
    if control == W.CTRL_TORQUE:
        w = W.fp_torque(seed=41, n_worlds=100, steps=200)
        w.ctrl_every = 4
    else:
        w = W.fp_position(seed=42, n_worlds=100, steps=500)
        w.ctrl_every = 5
    sim = _sim(w, B.F_WORKQUEUE)
    x = dev(w.x0)
    sim.step_k(x, dev(w.cmds), w.steps)
    torch.cuda.synchronize()
    assert_states_close(x, O.simulate_held(w), w, what=f"control {control} every {w.ctrl_every}")


@pytest.mark.parametrize("K", [1, 3, 6])
def test_rollout_gradients_slow_pid(gpu_lib, K):
    """Mixed first-principles (PID every 3 steps) and identified worlds, 100 steps
    (the last block is one step long), checkpoints every K steps (K divides the
    block or the block divides K): loss, x_T and gradients vs autograd."""
    w = W.uneven_mixed_adjoint(seed=9, n_worlds=12, n_subset=8, steps=100, n_max=70)
    w.ctrl_every = 3
    _check_against_oracle(w, _rollout_grads(w, K))


def test_rollout_gradients_slow_torque_allocation(gpu_lib):
    w = _torque_rollout_workload(90, aero=False)
    w.ctrl_every = 4
    _check_against_oracle(w, _rollout_grads(w, 2))


def test_sampled_rollouts_with_slow_controller(gpu_lib):
    """Controller every 2 of 4 physics steps per horizon step (5 ms physics)."""
    w, P, mean0 = W.mppi_task(n_controllers=2, n_samples=600, horizon=11, dt=0.005, substeps=4)
    w.ctrl_every = 2
    P["n_elite"] = 12
    sim = _sim(w)
    mp = B.Mppi(sim, P)
    C, N = P["n_controllers"], P["n_samples"]
    cost = torch.empty((C, N), device="cuda")
    mp.step(dev(w.x0[:, 0]), dev(mean0), 0, 3, cost=cost)
    torch.cuda.synchronize()
    cc, kk = np.repeat(np.arange(C), N), np.tile(np.arange(N), C)
    eps = OM.correlated_noise(cc, kk, P["horizon"], P["seed"], 3, P["beta"])
    u = OM.sample_commands(OM.shifted_mean(mean0.astype(np.float64), 0), cc, eps, P)
    Jr = OM.rollout_costs(w, w.x0[:, 0], u, P)
    Jg = cost.cpu().numpy()[cc, kk].astype(np.float64)
    assert np.max(np.abs(Jg - Jr) / np.abs(Jr)) <= 1e-4
    mp.close()


def test_rejects_step_counts_and_intervals_off_the_block(gpu_lib):
    w = W.uneven_mixed_adjoint(seed=9, n_worlds=4, n_subset=3, steps=12, n_max=20)
    w.ctrl_every = 3
    sim = _sim(w)
    x = dev(w.x0)
    u = dev(w.cmds[0])
    with pytest.raises(B.CfError):
        sim.step_k(x, u, 4)
    T, K = w.steps, 2
    ckpt = sim.ckpt_buffer(T, K)
    with pytest.raises(B.CfError):
        sim.rollout(x, dev(w.cmds), T, None, K, ckpt=ckpt)
    sim.step_k(x, u, 6)   # a multiple of the block is accepted
    torch.cuda.synchronize()
