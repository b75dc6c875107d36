"""The BPTT reward objective (CF_OBJ_BPTT_REWARD) through the C ABI vs the FP64
oracle: loss, final state and gradients for the identified and PID models with
feedback, checkpoint intervals 1 and 10, hover on the reference, the argument
checks, and BPTT on the paper's weights."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_helpers import dev
from paper_2606_01478_amd import binding as B
from paper_2606_01478_amd.bptt import train_linear_policy
from test_gpu_parity import _check_against_oracle, _rollout_grads
from test_oracle_pins import _hover_on_reference, _tilted

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K", [1, 10])
def test_reward_gradients_identified(gpu_lib, K):
    w = W.small("id_rollout_grad", seed=31)
    w.reward = W.BPTT_REWARD
    _check_against_oracle(_tilted(w, 31), _rollout_grads(w, K))


@pytest.mark.parametrize("K", [1, 10])
def test_reward_gradients_mixed_pid(gpu_lib, K):
    w = W.uneven_mixed_adjoint(seed=32, n_worlds=12, n_subset=8, steps=120, n_max=70)
    w.reward = W.BPTT_REWARD
    w = _tilted(w, 32)
    _check_against_oracle(w, _rollout_grads(w, K))


def test_reward_torque_interface(gpu_lib):
    from test_gpu_parity import _torque_rollout_workload
    w = _torque_rollout_workload(33, aero=False)
    w.reward = dict(w_tilt=0.1, w_act=[100.0, 1e6, 1e6, 1e6], w_dact=[10.0, 1e7, 1e7, 1e7])
    _check_against_oracle(_tilted(w, 33), _rollout_grads(w, 4))


def test_reward_one_per_step_in_hover(gpu_lib):
    w = W.id_rollout_grad(seed=7, n_worlds=70, steps=30)
    w.x0[6:9] = 0.0
    w.x0[3:6] = 0.0
    w.x0[12] = W.MASS * W.GRAVITY / W.ID_CF
    w = _hover_on_reference(w)
    w.reward = W.BPTT_REWARD
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    loss = torch.empty(sim.D, device="cuda")
    obj = B.Sim.objective(ref_amp=0.0, ref_period=w.ref_period, ref_offset=dev(w.ref_offset), reward=w.reward)
    ckpt = sim.ckpt_buffer(w.steps, 10, B.CF_OBJ_BPTT_REWARD)
    sim.rollout(dev(w.x0), dev(w.cmds), w.steps, obj, 10, ckpt=ckpt, loss=loss)
    torch.cuda.synchronize()
    assert np.allclose(loss.cpu().numpy(), -w.steps, rtol=0, atol=1e-4 * w.steps)


def test_reward_rejects_position_interface_and_bad_weights(gpu_lib):
    w = W.fp_position(seed=34, n_worlds=4, steps=10)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    x0 = dev(w.x0)
    cmds = dev(np.repeat(w.cmds[None], 10, 0))
    ckpt = sim.ckpt_buffer(10, 10, B.CF_OBJ_BPTT_REWARD)
    with pytest.raises(B.CfError):
        sim.rollout(x0, cmds, 10, B.Sim.objective(reward=W.BPTT_REWARD), 10, ckpt=ckpt)
    w2 = W.small("id_rollout_grad", seed=35)
    sim2 = B.Sim.from_workload(w2, flags=B.F_NO_AUTOTUNE_CACHE)
    bad = dict(W.BPTT_REWARD, w_tilt=-1.0)
    ck2 = sim2.ckpt_buffer(w2.steps, 10, B.CF_OBJ_BPTT_REWARD)
    with pytest.raises(B.CfError):
        sim2.rollout(dev(w2.x0), dev(w2.cmds), w2.steps, B.Sim.objective(reward=bad), 10, ckpt=ck2)


def test_bptt_on_the_paper_reward(gpu_lib):
    """16 environments, 40-step rollouts, the paper's weights and learning rate:
    the summed reward rises."""
    w = W.id_rollout_grad(seed=36, n_worlds=16, steps=40)
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, reward=W.BPTT_REWARD)
    out = train_linear_policy(sim, dev(w.x0), dev(w.cmds), w.steps, dev(w.gain), iters=60, lr=4.6e-2,
                              ckpt_every=10, obj_kw=kw, train_commands=True)
    torch.cuda.synchronize()
    losses = out["losses"].cpu().numpy()
    assert np.all(np.isfinite(losses))
    # the start is already close to the reference (reward about 0.85 per step of
    # a maximum of 1), so the gain is modest: the reward ends higher than it began
    assert losses[-1] < losses[0] - 0.004 * abs(losses[0]), (losses[0], losses[-1])


def test_reward_with_slow_controller(gpu_lib):
    """The reward objective and a PID running every third step together
    (checkpoint interval 3)."""
    w = W.uneven_mixed_adjoint(seed=37, n_worlds=10, n_subset=6, steps=61, n_max=50)
    w.reward = W.BPTT_REWARD
    w.ctrl_every = 3
    w = _tilted(w, 37)
    _check_against_oracle(w, _rollout_grads(w, 3))
