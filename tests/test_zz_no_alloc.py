"""The allocation-free backward (cf_rollout_backward_noalloc) against the
allocating one (cf_rollout_backward) through the C ABI: bit-identical
gradients on two calls in a row, the second on a smaller input (the static
scratch still holds the first call's contents), and a request whose scratch
exceeds the static array refused with CF_EINVAL before any work."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import dev
from paper_2606_01478_amd import binding as B

pytestmark = pytest.mark.gpu


def _grads(sim, w, K, noalloc):
    T = w.steps
    x0, cmds = dev(w.x0), dev(w.cmds)
    gain = None if w.gain is None else dev(w.gain)
    off = None if w.ref_offset is None else dev(w.ref_offset)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, ref_offset=off, w_u=w.w_u,
                          reward=w.reward)
    ckpt = sim.ckpt_buffer(T, K, int(obj.kind))
    sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt)
    g = (torch.full_like(cmds, 7.0), torch.full_like(x0, 7.0), None if gain is None else torch.full_like(gain, 7.0))
    back = sim.rollout_backward_noalloc if noalloc else sim.rollout_backward
    back(x0, cmds, T, obj, K, ckpt, dloss=dev(w.dloss), g_cmds=g[0], g_x0=g[1], g_gain=g[2])
    torch.cuda.synchronize()
    return g


def test_noalloc_backward_equals_the_allocating_backward(gpu_lib):
    big = W.uneven_mixed_adjoint(seed=96, n_worlds=24, n_subset=12, steps=150, n_max=300)   # both models, 2 gains
    small = W.id_rollout_grad(seed=97, n_worlds=90, steps=40)                                     # fewer drones, shorter
    small.reward = W.BPTT_REWARD
    for w, K in ((big, 40), (small, 10)):
        sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
        ref = _grads(sim, w, K, noalloc=False)
        got = _grads(sim, w, K, noalloc=True)
        for a, b, name in zip(got, ref, ("g_cmds", "g_x0", "g_gain")):
            if b is not None:
                assert torch.isfinite(b).all(), name
                assert torch.equal(a, b), name
        assert sim.last_error() == 0
        sim.close()


def test_noalloc_backward_refuses_scratch_beyond_the_static_array(gpu_lib):
    w = W.id_rollout_grad(seed=98, n_worlds=70000, steps=200)   # 100 segment slots x 13 rows x 70 000 drones
    sim = B.Sim.from_workload(w, flags=B.F_NO_AUTOTUNE_CACHE)
    T, K = w.steps, 100
    x0, cmds, gain = dev(w.x0), dev(w.cmds), dev(w.gain)
    obj = B.Sim.objective(gain=gain, ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    ckpt = sim.ckpt_buffer(T, K)
    sim.rollout(x0, cmds, T, obj, K, ckpt=ckpt)
    g = torch.full_like(cmds, 7.0)
    st = sim._lib.cf_rollout_backward_noalloc(sim._h, x0.data_ptr(), cmds.data_ptr(), T, ctypes.byref(obj), K,
                                              ckpt.data_ptr(), None, g.data_ptr(), None, None)
    assert st == B.CF_EINVAL
    torch.cuda.synchronize()
    assert (g == 7.0).all()           # nothing written
    # the allocating backward of the same request works
    sim.rollout_backward(x0, cmds, T, obj, K, ckpt, g_cmds=g)
    torch.cuda.synchronize()
    assert torch.isfinite(g).all() and sim.last_error() == 0
