"""Shared helpers of the GPU parity tests (tolerances, device transfer, sampling)."""
import dataclasses
import json
import os

import numpy as np
import torch

import workloads as W

# Parity bar on states (FP32 device vs FP64 oracle): per component
# |x_gpu - x_ref| <= 1e-4 * max(|x_ref|, floor), with the floors below.
STATE_RTOL = 1e-4
GRAD_RTOL = 1e-3
HOVER_SPEED = float(W.hover_speed(W.MASS))


def log_margin(what, ratio):
    """Append the worst error/bound ratio of a check to $CFSIM_PARITY_LOG (if set)."""
    path = os.environ.get("CFSIM_PARITY_LOG")
    if path:
        test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
        with open(path, "a") as f:
            f.write(json.dumps({"test": test, "check": what, "max_err_over_bound": ratio}) + "\n")


def state_floors(S: int, model_rows=None) -> np.ndarray:
    """Floors per state row: position 1 m, attitude 1, velocity 1 m/s, body rate
    1 rad/s, rotor speed = hover speed, controller state 1; identified model:
    angle 1 rad, angle rate 1 rad/s, thrust state m g."""
    if S == W.S_ID:
        f = np.ones(S)
        f[12] = W.MASS * W.GRAVITY
        return f
    f = np.ones(S)
    f[13:17] = HOVER_SPEED
    return f


def floors_for(w) -> np.ndarray:
    """[S, D] floors (mixed handles: identified drones use the identified floors)."""
    S, D = w.x0.shape
    fl = np.broadcast_to(state_floors(S)[:, None], (S, D)).copy()
    world = np.repeat(np.arange(w.n_worlds), w.drones_per_world)
    idm = w.model_per_world[world] == W.MODEL_ID
    if idm.any():
        fl[:13, idm] = state_floors(W.S_ID)[:, None]
    return fl


def assert_states_close(gpu, ref, w, rows=None, what="state"):
    gpu = gpu.detach().cpu().double().numpy() if isinstance(gpu, torch.Tensor) else np.asarray(gpu, np.float64)
    ref = ref.detach().cpu().double().numpy() if isinstance(ref, torch.Tensor) else np.asarray(ref, np.float64)
    fl = floors_for(w)
    world = np.repeat(np.arange(w.n_worlds), w.drones_per_world)
    mask = np.ones_like(ref, dtype=bool)
    if w.x0.shape[0] > W.S_ID:
        idm = w.model_per_world[world] == W.MODEL_ID
        mask[W.S_ID:, idm] = False         # rows unused by identified drones
    bound = STATE_RTOL * np.maximum(np.abs(ref), fl)
    err = np.abs(gpu - ref)
    bad = (err > bound) & mask
    assert np.isfinite(gpu[mask]).all(), f"{what}: non-finite values"
    if bad.any():
        i, d = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} components out of tolerance; first row {i} drone {d}: "
                             f"gpu {gpu[i, d]!r} ref {ref[i, d]!r} bound {bound[i, d]!r}; "
                             f"max err/bound {(err / bound)[mask].max():.3g}")
    r = float((err / bound)[mask].max())
    log_margin(what, r)
    return r


def assert_grad_close(gpu, ref, what, axis_drone=-1):
    """Per drone (block over every other axis): |g - g_ref|_2 <= 1e-3 |g_ref|_2."""
    g = gpu.detach().cpu().double().numpy()
    r = ref.detach().cpu().double().numpy()
    g2 = np.moveaxis(g, axis_drone, 0).reshape(g.shape[axis_drone], -1)
    r2 = np.moveaxis(r, axis_drone, 0).reshape(r.shape[axis_drone], -1)
    num = np.linalg.norm(g2 - r2, axis=1)
    den = np.linalg.norm(r2, axis=1)
    ok = num <= GRAD_RTOL * np.maximum(den, 1e-12)
    if not ok.all():
        d = int(np.argmin(ok))
        raise AssertionError(f"{what}: {(~ok).sum()} drones out of tolerance; drone {d}: rel {num[d] / den[d]:.3g}")
    r = float((num / np.maximum(den, 1e-30)).max()) / GRAD_RTOL
    log_margin(what, r)
    return r


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dtype).contiguous()


def sample_drones(w, idx):
    """Workload of single-drone worlds for the given global drone indices (each
    with its world's parameters, model and gain index) -- drones never interact,
    so the oracle can check them one by one."""
    idx = np.asarray(idx)
    world = np.repeat(np.arange(w.n_worlds), w.drones_per_world)[idx]
    n = len(idx)
    return dataclasses.replace(
        w, n_worlds=n, drones_per_world=np.ones(n, np.int32), model_per_world=w.model_per_world[world].copy(),
        params={k: v[world].copy() for k, v in w.params.items()}, x0=np.ascontiguousarray(w.x0[:, idx]),
        cmds=np.ascontiguousarray(w.cmds[..., idx]),
        gain_index=None if w.gain_index is None else w.gain_index[world].copy(),
        ref_offset=None if w.ref_offset is None else np.ascontiguousarray(w.ref_offset[:, idx]),
        dloss=None if w.dloss is None else w.dloss[idx].copy())
