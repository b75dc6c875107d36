"""ctypes binding of libcfsim.so (include/cfsim.h).

Argument marshalling only: every step of the simulation runs in the HIP
library. PyTorch supplies device memory (CUDA/HIP tensors) and the stream.
Loading fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_uint8, c_uint32, c_void_p
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfsim.so")

CF_OK, CF_EINVAL, CF_ENODEV, CF_ENOMEM, CF_EDEVICE, CF_ESTATE, CF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MODEL_FP, MODEL_ID = 0, 1
CTRL_ROTOR, CTRL_ATT_PID, CTRL_TORQUE, CTRL_POSITION = 0, 1, 2, 3
INTEG_EULER, INTEG_RK4 = 0, 1
F_PLAIN_KERNEL, F_NONFINITE_CHECK, F_GRAPH, F_WORKQUEUE, F_NO_AUTOTUNE_CACHE = 0x1, 0x2, 0x4, 0x8, 0x10
F_SINGLE_LAUNCH = 0x20
F_TIMING = 0x40
CF_OBJ_TRACKING, CF_OBJ_BPTT_REWARD = 0, 1
S_FP_ROTOR, S_FP_PID, S_ID = 17, 25, 13
NPARAM = 96
NGAIN = 52

# offsets of the named parameter fields in the CF_NPARAM record (CF_P_* in the header)
PARAM_OFFSETS = {
    "mass": (0, 1), "gravity": (1, 1), "J": (2, 3), "thrust_poly": (5, 3), "torque_poly": (8, 3),
    "mix_tx": (11, 4), "mix_ty": (15, 4), "mix_yaw": (19, 4), "motor_up": (23, 2), "motor_down": (25, 2),
    "Jp": (27, 1), "drag": (28, 3), "ang_kp": (31, 2), "ang_ki": (33, 2), "rate_kp": (35, 3),
    "rate_ki": (38, 3), "rate_kd": (41, 3), "J_ctrl": (44, 3), "f_max": (47, 1), "alloc": (48, 16),
    "c_f": (64, 1), "c_tau": (65, 1), "c_psi1": (66, 3), "c_psi2": (69, 3), "c_psi3": (72, 3),
    "pos_kp": (75, 3), "pos_kv": (78, 3), "att_kr": (81, 3), "att_kw": (84, 3),
}

EXPORTS = ("cf_create", "cf_destroy", "cf_state_dim", "cf_total_drones", "cf_world_offsets", "cf_set_stream",
           "cf_reset", "cf_step_k", "cf_rollout", "cf_rollout_backward", "cf_rollout_backward_noalloc", "cf_ckpt_floats", "cf_autotune", "cf_launch_config", "cf_set_launch_config", "cf_launch_times",
           "cf_strerror", "cf_last_error", "cf_mppi_create", "cf_mppi_destroy", "cf_mppi_step", "cf_mppi_noise", "cf_probe_fma")

MPPI_MAX_OBSTACLES = 16
MPPI_MAX_ELITE = 4096


class CfError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_LIB.cf_strerror(status).decode() if _LIB else status} ({status})")


class _Desc(ctypes.Structure):
    _fields_ = [("n_worlds", c_int32), ("n_drones", c_int32), ("drones_per_world", POINTER(c_int32)),
                ("model", c_int32), ("model_per_world", POINTER(c_uint8)), ("control", c_int32),
                ("integrator", c_int32), ("dt", c_float), ("renorm_q", c_int32), ("params", POINTER(c_float)),
                ("n_gains", c_int32), ("gain_index", POINTER(c_int32)), ("stream", c_void_p),
                ("flags", c_uint32), ("device", c_int32), ("ctrl_every", c_int32)]


class _Objective(ctypes.Structure):
    _fields_ = [("gain", c_void_p), ("ref_table", c_void_p), ("ref_amp", c_float), ("ref_period", c_float),
                ("ref_offset", c_void_p), ("w_u", c_float), ("kind", c_int32), ("w_tilt", c_float),
                ("w_act", c_float * 4), ("w_dact", c_float * 4), ("policy_hidden", c_int32),
                ("ref_step0", c_int32),
                ("ref_time_shift", c_void_p), ("policy_scale", c_float * 4)]


class _MppiDesc(ctypes.Structure):
    _fields_ = [("n_controllers", c_int32), ("n_samples", c_int32), ("horizon", c_int32), ("substeps", c_int32),
                ("n_elite", c_int32), ("sigma", c_float * 4), ("beta", c_float), ("lambda_", c_float),
                ("u_lo", c_float * 4), ("u_hi", c_float * 4), ("u_ref", c_float * 4), ("r_u", c_float * 4),
                ("goal", c_float * 3), ("q_p", c_float), ("q_v", c_float), ("w_obs", c_float),
                ("n_obstacles", c_int32), ("obstacles", (c_float * 4) * MPPI_MAX_OBSTACLES),
                ("seed", ctypes.c_uint64)]


_LIB: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2606_01478_amd.build.build()")
    lib = ctypes.CDLL(path)
    H = c_void_p
    P = c_void_p
    sig = {
        "cf_create": ([POINTER(_Desc), POINTER(c_void_p)], c_int32),
        "cf_destroy": ([H], c_int32),
        "cf_state_dim": ([H, POINTER(c_int32)], c_int32),
        "cf_total_drones": ([H, POINTER(c_int64)], c_int32),
        "cf_world_offsets": ([H, POINTER(c_int64)], c_int32),
        "cf_set_stream": ([H, c_void_p], c_int32),
        "cf_reset": ([H, P, P, P], c_int32),
        "cf_step_k": ([H, P, P, c_int32, P], c_int32),
        "cf_rollout": ([H, P, P, c_int32, POINTER(_Objective), c_int32, P, P, P, P, P], c_int32),
        "cf_rollout_backward": ([H, P, P, c_int32, POINTER(_Objective), c_int32, P, P, P, P, P], c_int32),
        "cf_rollout_backward_noalloc": ([H, P, P, c_int32, POINTER(_Objective), c_int32, P, P, P, P, P], c_int32),
        "cf_ckpt_floats": ([H, c_int32, c_int32, c_int32, POINTER(c_int64)], c_int32),
        "cf_autotune": ([H, P, P, c_int32, c_int32], c_int32),
        "cf_launch_config": ([H, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)], c_int32),
        "cf_set_launch_config": ([H, c_int32, c_int32, c_int32, c_int32], c_int32),
        "cf_launch_times": ([H, c_int32, POINTER(c_float), c_int32, POINTER(c_int32)], c_int32),
        "cf_strerror": ([c_int32], ctypes.c_char_p),
        "cf_last_error": ([H], c_int32),
        "cf_mppi_create": ([H, POINTER(_MppiDesc), POINTER(c_void_p)], c_int32),
        "cf_mppi_destroy": ([H], c_int32),
        "cf_mppi_step": ([H, P, P, c_int32, ctypes.c_uint64, P, P, P, P, P], c_int32),
        "cf_mppi_noise": ([H, ctypes.c_uint64, P], c_int32),
        "cf_probe_fma": ([P, c_int32, c_int32, c_int32, c_void_p], c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def _check(status: int, what: str) -> None:
    if status != CF_OK:
        raise CfError(status, what)


def mlp_params(hidden: int) -> int:
    """Floats of one small-MLP policy of width ``hidden`` (CF_MLP_PARAMS in the C header)."""
    H = int(hidden)
    return 13 * H + H + H * H + H + 4 * H + 4


def pack_params(params: Dict[str, np.ndarray], n_worlds: int) -> np.ndarray:
    """Named per-world fields ``[M, k]`` -> the flat ``[M][CF_NPARAM]`` float32 record."""
    out = np.zeros((n_worlds, NPARAM), np.float32)
    for name, arr in params.items():
        off, k = PARAM_OFFSETS[name]
        a = np.asarray(arr, np.float32).reshape(n_worlds, k)
        out[:, off:off + k] = a
    return out


def _ptr(t) -> Optional[int]:
    """Device address of a contiguous float32/uint8/uint32 CUDA tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


class Sim:
    """A batch of worlds on one GPU (handle of the C library)."""

    def __init__(self, n_worlds: int, drones_per_world, model_per_world, control: int, integrator: int,
                 dt: float, params, *, renorm_q: int = 1, n_gains: int = 0, gain_index=None, flags: int = 0,
                 device: int = -1, ctrl_every: int = 1):
        import torch
        lib = load()
        self._lib = lib
        self._h = c_void_p()
        M = int(n_worlds)
        self.n_worlds = M
        counts = np.ascontiguousarray(np.broadcast_to(np.asarray(drones_per_world, np.int32), (M,)))
        models = np.ascontiguousarray(np.broadcast_to(np.asarray(model_per_world, np.uint8), (M,)))
        flat = pack_params(params, M) if isinstance(params, dict) else np.ascontiguousarray(params, np.float32)
        if flat.shape != (M, NPARAM):
            raise ValueError(f"params must be [{M}, {NPARAM}]")
        self._keep = [counts, models, flat]
        d = _Desc()
        d.n_worlds = M
        d.n_drones = 0
        d.drones_per_world = counts.ctypes.data_as(POINTER(c_int32))
        d.model = int(models[0]) if M else 0
        d.model_per_world = models.ctypes.data_as(POINTER(c_uint8))
        d.control = int(control)
        d.integrator = int(integrator)
        d.dt = float(dt)
        d.renorm_q = int(renorm_q)
        d.params = flat.ctypes.data_as(POINTER(c_float))
        d.n_gains = int(n_gains)
        if gain_index is not None:
            gi = np.ascontiguousarray(np.asarray(gain_index, np.int32).reshape(M))
            self._keep.append(gi)
            d.gain_index = gi.ctypes.data_as(POINTER(c_int32))
        d.stream = c_void_p(_stream() if torch.cuda.is_available() else 0)
        d.flags = int(flags)
        d.device = int(device)
        d.ctrl_every = int(ctrl_every)
        _check(lib.cf_create(ctypes.byref(d), ctypes.byref(self._h)), "cf_create")
        S = c_int32()
        D = c_int64()
        _check(lib.cf_state_dim(self._h, ctypes.byref(S)), "cf_state_dim")
        _check(lib.cf_total_drones(self._h, ctypes.byref(D)), "cf_total_drones")
        self.S, self.D = int(S.value), int(D.value)
        off = np.zeros(M + 1, np.int64)
        _check(lib.cf_world_offsets(self._h, off.ctypes.data_as(POINTER(c_int64))), "cf_world_offsets")
        self.offsets = off
        self.n_gains = int(n_gains)
        self.flags = int(flags)
        self.ctrl_every = int(ctrl_every)

    @classmethod
    def from_workload(cls, w, flags: int = 0, **kw):
        n_gains = 0 if w.gain is None else int(w.gain.shape[0])
        kw.setdefault("ctrl_every", getattr(w, "ctrl_every", 1))
        return cls(w.n_worlds, w.drones_per_world, w.model_per_world, w.control, w.integrator, w.dt,
                   w.params, renorm_q=w.renorm_q, n_gains=n_gains, gain_index=w.gain_index, flags=flags, **kw)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.cf_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _need(self, t, shape, name, dtypes=("float32",)) -> None:
        if t is None:
            return
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        if str(t.dtype).replace("torch.", "") not in dtypes:
            raise ValueError(f"{name}: expected dtype {dtypes}, got {t.dtype}")

    def _gain_shape(self, obj):
        """Shape of the feedback parameters: linear gains or small-MLP policies."""
        if obj is not None and obj.policy_hidden > 0:
            return (self.n_gains, mlp_params(obj.policy_hidden))
        return (self.n_gains, 4, 13)

    def _need_obj(self, obj, T) -> None:
        if obj is None:
            return
        g, rt, ro, rs = getattr(obj, "_tensors", (None, None, None, None))
        self._need(g, self._gain_shape(obj), "gain")
        self._need(rt, (T + 1, 13), "ref_table")
        self._need(ro, (3, self.D), "ref_offset")
        self._need(rs, (self.D,), "ref_time_shift")

    def _sync_stream(self) -> None:
        _check(self._lib.cf_set_stream(self._h, c_void_p(_stream())), "cf_set_stream")

    # -- calls -------------------------------------------------------------------
    def reset(self, state, init, world_mask=None) -> None:
        self._need(state, (self.S, self.D), "state")
        self._need(init, (self.S, self.D), "init")
        self._need(world_mask, (self.n_worlds,), "world_mask", ("uint8", "bool"))
        self._sync_stream()
        _check(self._lib.cf_reset(self._h, _ptr(state), _ptr(init), _ptr(world_mask)), "cf_reset")

    def step_k(self, state, cmd, k: int, nonfinite=None) -> None:
        self._need(state, (self.S, self.D), "state")
        self._need(cmd, (4, self.D), "cmd")
        self._need(nonfinite, (self.n_worlds,), "nonfinite", ("int32", "uint32"))
        self._sync_stream()
        _check(self._lib.cf_step_k(self._h, _ptr(state), _ptr(cmd), int(k), _ptr(nonfinite)), "cf_step_k")

    @staticmethod
    def objective(gain=None, ref_table=None, ref_amp=1.0, ref_period=4.0, ref_offset=None, w_u=1e-3,
                  reward=None, policy_hidden=0, ref_step0=0, ref_time_shift=None, policy_scale=None):
        """Tracking objective; with ``reward`` = dict(w_tilt, w_act[4], w_dact[4]) the
        BPTT reward objective (CF_OBJ_BPTT_REWARD) instead. With ``policy_hidden`` = H
        > 0, ``gain`` holds small-MLP policies [n_gains, mlp_params(H)] instead of
        linear gains [n_gains, 4, 13]. ``ref_time_shift`` [D] (seconds) moves each
        drone's point on the figure-eight. ``policy_scale`` (4 floats) squashes the
        policy output o into ``policy_scale * tanh(o)``."""
        o = _Objective()
        o.policy_hidden = int(policy_hidden)
        o.ref_step0 = int(ref_step0)
        o.gain = _ptr(gain)
        o.ref_table = _ptr(ref_table)
        o.ref_amp = float(ref_amp)
        o.ref_period = float(ref_period)
        o.ref_offset = _ptr(ref_offset)
        o.ref_time_shift = _ptr(ref_time_shift)
        if policy_scale is not None:
            for i in range(4):
                o.policy_scale[i] = float(policy_scale[i])
        o.w_u = float(w_u)
        if reward is not None:
            o.kind = CF_OBJ_BPTT_REWARD
            o.w_tilt = float(reward["w_tilt"])
            for i in range(4):
                o.w_act[i] = float(reward["w_act"][i])
                o.w_dact[i] = float(reward["w_dact"][i])
        o._tensors = (gain, ref_table, ref_offset, ref_time_shift)
        return o

    def ckpt_floats(self, T: int, ckpt_every: int, kind: int = CF_OBJ_TRACKING) -> int:
        """Floats of the checkpoint buffer of a rollout (states every ``ckpt_every``
        steps, the reward objective's applied commands, the forward's tag)."""
        n = c_int64()
        _check(self._lib.cf_ckpt_floats(self._h, int(T), int(ckpt_every), int(kind), ctypes.byref(n)),
               "cf_ckpt_floats")
        return int(n.value)

    def ckpt_buffer(self, T: int, ckpt_every: int, kind: int = CF_OBJ_TRACKING, device="cuda"):
        """A device buffer for the checkpoints of a rollout (flat float32)."""
        import torch
        return torch.empty(self.ckpt_floats(T, ckpt_every, kind), device=device, dtype=torch.float32)

    def ckpt_states(self, ckpt, T: int, ckpt_every: int):
        """View of the checkpoint states inside a checkpoint buffer, ``[ceil(T/K), S, D]``."""
        nseg = (int(T) + int(ckpt_every) - 1) // int(ckpt_every)
        return ckpt[:nseg * self.S * self.D].view(nseg, self.S, self.D)

    def _need_ckpt(self, ckpt, T, ckpt_every, obj) -> None:
        if ckpt is None:
            return
        kind = CF_OBJ_TRACKING if obj is None else int(obj.kind)
        n = self.ckpt_floats(T, ckpt_every, kind)
        if ckpt.dim() != 1 or ckpt.numel() != n or str(ckpt.dtype) != "torch.float32":
            raise ValueError(f"ckpt: expected a flat float32 buffer of {n} values (Sim.ckpt_buffer), "
                             f"got {tuple(ckpt.shape)} {ckpt.dtype}")

    def rollout(self, x0, cmds, T: int, obj=None, ckpt_every: int = 50, ckpt=None, x_T=None, traj=None,
                loss=None, loss_world=None) -> None:
        T = int(T)
        self._need(x0, (self.S, self.D), "x0")
        self._need(cmds, (T, 4, self.D), "cmds")
        self._need_ckpt(ckpt, T, ckpt_every, obj)
        self._need(x_T, (self.S, self.D), "x_T")
        self._need(traj, (T + 1, self.S, self.D), "traj")
        self._need(loss, (self.D,), "loss")
        self._need(loss_world, (self.n_worlds,), "loss_world")
        self._need_obj(obj, T)
        self._sync_stream()
        o = ctypes.byref(obj) if obj is not None else None
        _check(self._lib.cf_rollout(self._h, _ptr(x0), _ptr(cmds), int(T), o, int(ckpt_every), _ptr(ckpt),
                                    _ptr(x_T), _ptr(traj), _ptr(loss), _ptr(loss_world)), "cf_rollout")

    def rollout_backward(self, x0, cmds, T: int, obj, ckpt_every: int, ckpt, dloss=None, g_cmds=None,
                         g_x0=None, g_gain=None) -> None:
        T = int(T)
        self._need(cmds, (T, 4, self.D), "cmds")
        self._need_ckpt(ckpt, T, ckpt_every, obj)
        self._need(dloss, (self.D,), "dloss")
        self._need(g_cmds, (T, 4, self.D), "g_cmds")
        self._need(g_x0, (self.S, self.D), "g_x0")
        self._need(g_gain, self._gain_shape(obj), "g_gain")
        self._need_obj(obj, T)
        self._sync_stream()
        o = ctypes.byref(obj) if obj is not None else None
        _check(self._lib.cf_rollout_backward(self._h, _ptr(x0), _ptr(cmds), int(T), o, int(ckpt_every),
                                             _ptr(ckpt), _ptr(dloss), _ptr(g_cmds), _ptr(g_x0), _ptr(g_gain)),
               "cf_rollout_backward")

    def rollout_backward_noalloc(self, x0, cmds, T: int, obj, ckpt_every: int, ckpt, dloss=None, g_cmds=None,
                                 g_x0=None, g_gain=None) -> None:
        """rollout_backward without device allocation (scratch in the library's
        static per-GPU array; calls on one GPU must not overlap)."""
        T = int(T)
        self._need(cmds, (T, 4, self.D), "cmds")
        self._need_ckpt(ckpt, T, ckpt_every, obj)
        self._need(dloss, (self.D,), "dloss")
        self._need(g_cmds, (T, 4, self.D), "g_cmds")
        self._need(g_x0, (self.S, self.D), "g_x0")
        self._need(g_gain, self._gain_shape(obj), "g_gain")
        self._need_obj(obj, T)
        self._sync_stream()
        o = ctypes.byref(obj) if obj is not None else None
        _check(self._lib.cf_rollout_backward_noalloc(self._h, _ptr(x0), _ptr(cmds), int(T), o, int(ckpt_every),
                                                     _ptr(ckpt), _ptr(dloss), _ptr(g_cmds), _ptr(g_x0),
                                                     _ptr(g_gain)), "cf_rollout_backward_noalloc")

    def autotune(self, state, cmd, k: int, budget_ms: int = 2000) -> None:
        self._need(state, (self.S, self.D), "state")
        self._need(cmd, (4, self.D), "cmd")
        self._sync_stream()
        _check(self._lib.cf_autotune(self._h, _ptr(state), _ptr(cmd), int(k), int(budget_ms)), "cf_autotune")

    def launch_config(self):
        a, b, c = c_int32(), c_int32(), c_int32()
        _check(self._lib.cf_launch_config(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "cf_launch_config")
        return {"workqueue": a.value & 1, "per_model_launches": (a.value >> 1) & 1, "tile": b.value, "chunk": c.value}

    def set_launch_config(self, workqueue: int = 0, tile: int = 64, chunk: int = 0, per_model_launches: int = 1,
                          wq_waves: int = 0):
        """Pin the launch choice of step_k (see launch_config); ``wq_waves`` caps the
        work queue's resident waves per compute unit (0 = as many as fit)."""
        wq = (int(workqueue) & 1) | ((int(per_model_launches) & 1) << 1)
        _check(self._lib.cf_set_launch_config(self._h, wq, int(tile), int(chunk), int(wq_waves)),
               "cf_set_launch_config")

    def launch_times(self, slot: int = 0):
        """Durations (ms) of the kernel launches of the latest step_k call on stream
        slot 0 or 1 (handles created with F_TIMING)."""
        buf = (c_float * 512)()
        n = c_int32()
        _check(self._lib.cf_launch_times(self._h, int(slot), buf, 512, ctypes.byref(n)), "cf_launch_times")
        return [float(buf[i]) for i in range(min(n.value, 512))]

    def last_error(self) -> int:
        return int(self._lib.cf_last_error(self._h))


def _rollout_loss_apply(sim: Sim, x0, cmds, gain, T, ckpt_every, obj_kw):
    import torch
    dev = x0.device
    obj = Sim.objective(gain=gain, **obj_kw)
    ckpt = sim.ckpt_buffer(T, ckpt_every, int(obj.kind), device=dev)
    loss = torch.empty(sim.D, device=dev, dtype=torch.float32)
    x_T = torch.empty_like(x0)
    sim.rollout(x0, cmds, T, obj, ckpt_every, ckpt=ckpt, x_T=x_T, loss=loss)
    return loss, ckpt, obj, x_T


class RolloutLoss:
    """``loss = RolloutLoss.apply(x0, cmds, gain, sim, T, ckpt_every, obj_kw)``: per-drone
    tracking loss ``[D]`` of a rollout; backward runs the library's discrete adjoint and
    returns gradients for ``x0`` ``[S][D]``, ``cmds`` ``[T][4][D]`` and ``gain``. Each
    application owns its checkpoint buffer (saved for its backward), so several
    applications on one handle may precede their backwards. With
    ``return_state=True`` it also returns the final state ``[S][D]`` (not
    differentiable), e.g. to start the next rollout from it."""

    @staticmethod
    def _fn():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, x0, cmds, gain, sim, T, ckpt_every, obj_kw):
                x0c, cmdsc = x0.detach().contiguous(), cmds.detach().contiguous()
                gc = None if gain is None else gain.detach().contiguous()
                loss, ckpt, _, x_T = _rollout_loss_apply(sim, x0c, cmdsc, gc, T, ckpt_every, obj_kw)
                ctx.sim, ctx.T, ctx.K, ctx.obj_kw = sim, T, ckpt_every, obj_kw
                ctx.save_for_backward(x0c, cmdsc, ckpt, *( [gc] if gc is not None else []))
                ctx.has_gain = gc is not None
                ctx.mark_non_differentiable(x_T)
                return loss, x_T

            @staticmethod
            def backward(ctx, dloss, dx_T=None):
                saved = ctx.saved_tensors
                x0, cmds, ckpt = saved[0], saved[1], saved[2]
                gain = saved[3] if ctx.has_gain else None
                sim = ctx.sim
                g_cmds = torch.empty_like(cmds)
                g_x0 = torch.empty_like(x0)
                g_gain = torch.empty_like(gain) if gain is not None else None
                obj = Sim.objective(gain=gain, **ctx.obj_kw)
                sim.rollout_backward(x0, cmds, ctx.T, obj, ctx.K, ckpt, dloss=dloss.contiguous(),
                                     g_cmds=g_cmds, g_x0=g_x0, g_gain=g_gain)
                return g_x0, g_cmds, g_gain, None, None, None, None

        return _F

    _cached = None

    @classmethod
    def apply(cls, x0, cmds, gain, sim, T, ckpt_every=50, obj_kw=None, return_state=False):
        if cls._cached is None:
            cls._cached = cls._fn()
        loss, x_T = cls._cached.apply(x0, cmds, gain, sim, T, ckpt_every, obj_kw or {})
        return (loss, x_T) if return_state else loss


def probe_fma(out, n_blocks: int, iters: int, form: int = 0) -> None:
    """Launch the FP32 FMA throughput probe on the current stream (16 * iters FLOP
    per lane, 256 lanes per block; form 0 three-operand, 1 accumulate form)."""
    if out.numel() < n_blocks * 256 or str(out.dtype) != "torch.float32":
        raise ValueError("out must hold n_blocks * 256 float32 values")
    _check(load().cf_probe_fma(_ptr(out), int(n_blocks), int(iters), int(form), c_void_p(_stream())),
           "cf_probe_fma")


class Mppi:
    """Sampled-rollout controllers (iCEM/MPPI hybrid) on the single world of ``sim``.
    ``params`` holds n_controllers, n_samples, horizon, substeps, n_elite, sigma,
    beta, lambda, u_lo, u_hi, u_ref, r_u, goal, q_p, q_v, w_obs, obstacles
    ``[n][4]`` (centre, radius) and seed."""

    def __init__(self, sim: Sim, params: Dict):
        self._lib = sim._lib
        self.sim = sim
        d = _MppiDesc()
        d.n_controllers = int(params["n_controllers"])
        d.n_samples = int(params["n_samples"])
        d.horizon = int(params["horizon"])
        d.substeps = int(params.get("substeps", 1))
        d.n_elite = int(params["n_elite"])
        for name in ("sigma", "u_lo", "u_hi", "u_ref", "r_u"):
            getattr(d, name)[:] = [float(v) for v in params[name]]
        d.goal[:] = [float(v) for v in params["goal"]]
        d.beta = float(params["beta"])
        d.lambda_ = float(params["lambda"])
        d.q_p, d.q_v, d.w_obs = float(params["q_p"]), float(params["q_v"]), float(params["w_obs"])
        obs = np.asarray(params.get("obstacles", np.zeros((0, 4))), np.float32).reshape(-1, 4)
        if len(obs) > MPPI_MAX_OBSTACLES:
            raise ValueError(f"at most {MPPI_MAX_OBSTACLES} obstacles")
        d.n_obstacles = len(obs)
        for o in range(len(obs)):
            d.obstacles[o][:] = [float(v) for v in obs[o]]
        d.seed = int(params["seed"]) & 0xFFFFFFFFFFFFFFFF
        self.C, self.N, self.H, self.n_elite = d.n_controllers, d.n_samples, d.horizon, d.n_elite
        self._m = c_void_p()
        _check(self._lib.cf_mppi_create(sim._h, ctypes.byref(d), ctypes.byref(self._m)), "cf_mppi_create")

    def close(self) -> None:
        if getattr(self, "_m", None) is not None and self._m.value:
            self._lib.cf_mppi_destroy(self._m)
            self._m = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, x_now, mean, shift: int, iteration: int, u_apply=None, best=None, cost=None, elite_idx=None,
             cost_min=None) -> None:
        """One control step; ``mean`` ``[C][H][4]`` is updated in place."""
        sim = self.sim
        sim._need(x_now, (sim.S,), "x_now")
        sim._need(mean, (self.C, self.H, 4), "mean")
        sim._need(u_apply, (4,), "u_apply")
        sim._need(best, (1,), "best", ("int32",))
        sim._need(cost, (self.C, self.N), "cost")
        sim._need(elite_idx, (self.C, self.n_elite), "elite_idx", ("int32",))
        sim._need(cost_min, (self.C,), "cost_min")
        _check(self._lib.cf_mppi_step(self._m, _ptr(x_now), _ptr(mean), int(shift), int(iteration), _ptr(u_apply),
                                      _ptr(best), _ptr(cost), _ptr(elite_idx), _ptr(cost_min)), "cf_mppi_step")

    def noise(self, iteration: int, eps) -> None:
        self.sim._need(eps, (self.C, self.N, self.H, 4), "eps")
        _check(self._lib.cf_mppi_noise(self._m, int(iteration), _ptr(eps)), "cf_mppi_noise")
