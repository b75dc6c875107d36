"""The C-ABI library without a GPU: it loads, exports every function that
include/cfsim.h declares, its layout constants agree with the binding, and
argument validation returns the documented status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2606_01478_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = open(os.path.join(ROOT, "include", "cfsim.h")).read()


@pytest.fixture(scope="module")
def lib():
    return B.load()


def declared_functions():
    body = re.sub(r"/\*.*?\*/", "", HEADER, flags=re.S)
    return sorted(set(re.findall(r"\b(cf_[a-z_]+)\s*\(", body)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 14
    assert set(names) == set(B.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_param_offsets_match_header():
    defs = dict((k, int(v)) for k, v in re.findall(r"#define (CF_P_[A-Z0-9_]+)\s+(\d+)", HEADER))
    names = {"mass": "CF_P_MASS", "gravity": "CF_P_GRAVITY", "J": "CF_P_J", "thrust_poly": "CF_P_THRUST",
             "torque_poly": "CF_P_TORQUE", "mix_tx": "CF_P_MIX_TX", "mix_ty": "CF_P_MIX_TY",
             "mix_yaw": "CF_P_MIX_YAW", "motor_up": "CF_P_MOTOR_UP", "motor_down": "CF_P_MOTOR_DOWN",
             "Jp": "CF_P_JP", "drag": "CF_P_DRAG", "ang_kp": "CF_P_ANG_KP", "ang_ki": "CF_P_ANG_KI",
             "rate_kp": "CF_P_RATE_KP", "rate_ki": "CF_P_RATE_KI", "rate_kd": "CF_P_RATE_KD",
             "J_ctrl": "CF_P_J_CTRL", "f_max": "CF_P_F_MAX", "alloc": "CF_P_ALLOC", "c_f": "CF_P_CF",
             "c_tau": "CF_P_CTAU", "c_psi1": "CF_P_CPSI1", "c_psi2": "CF_P_CPSI2", "c_psi3": "CF_P_CPSI3",
             "pos_kp": "CF_P_POS_KP", "pos_kv": "CF_P_POS_KV", "att_kr": "CF_P_ATT_KR", "att_kw": "CF_P_ATT_KW"}
    assert set(names) == set(B.PARAM_OFFSETS) == {n for n, _ in W.PARAM_FIELDS}
    for n, macro in names.items():
        assert B.PARAM_OFFSETS[n][0] == defs[macro], n
    widths = dict(W.PARAM_FIELDS)
    for n, (off, k) in B.PARAM_OFFSETS.items():
        assert k == widths[n]
    spans = sorted(B.PARAM_OFFSETS.values())
    for (o1, k1), (o2, _) in zip(spans, spans[1:]):
        assert o1 + k1 <= o2
    assert int(re.search(r"#define CF_NPARAM (\d+)", HEADER).group(1)) == B.NPARAM
    for macro, val in (("CF_S_FP_ROTOR", W.S_FP_ROTOR), ("CF_S_FP_PID", W.S_FP_PID), ("CF_S_ID", W.S_ID)):
        assert int(re.search(rf"#define {macro}\s+(\d+)", HEADER).group(1)) == val


def test_pack_params_places_fields():
    w = W.small("uneven_mixed", 1)
    flat = B.pack_params(w.params, w.n_worlds)
    assert flat.shape == (w.n_worlds, B.NPARAM) and flat.dtype == np.float32
    for n, (off, k) in B.PARAM_OFFSETS.items():
        assert np.array_equal(flat[:, off:off + k], w.params[n].reshape(w.n_worlds, k))


def _desc(w, **over):
    counts = np.array(w.drones_per_world, np.int32, copy=True)
    models = np.array(w.model_per_world, np.uint8, copy=True)
    flat = B.pack_params(w.params, w.n_worlds)
    d = B._Desc()
    d.n_worlds = w.n_worlds
    d.n_drones = 0
    d.drones_per_world = counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.model = 0
    d.model_per_world = models.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    d.control = w.control
    d.integrator = w.integrator
    d.dt = w.dt
    d.renorm_q = 1
    d.params = flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    d.n_gains = 0
    d.stream = None
    d.flags = B.F_NO_AUTOTUNE_CACHE
    d.device = -1
    for k, v in over.items():
        setattr(d, k, v)
    return d, (counts, models, flat)


def _create(lib, d):
    h = ctypes.c_void_p(123)
    st = lib.cf_create(ctypes.byref(d), ctypes.byref(h))
    if st == B.CF_OK:
        lib.cf_destroy(h)
    else:
        assert h.value is None
    return st


@pytest.mark.parametrize("field,value", [
    ("n_worlds", 0), ("control", 7), ("integrator", -1), ("dt", 0.0), ("dt", float("nan")),
    ("renorm_q", 3), ("n_gains", -1),
])
def test_create_rejects_invalid_fields(lib, field, value):
    d, keep = _desc(W.small("fp_pid_closed_loop", 1), **{field: value})
    assert _create(lib, d) == B.CF_EINVAL


def test_create_rejects_bad_counts_models_params(lib):
    w = W.small("uneven_mixed", 1)
    d, keep = _desc(w)
    keep[0][3] = -1
    assert _create(lib, d) == B.CF_EINVAL
    d, keep = _desc(w)
    keep[1][2] = 9
    assert _create(lib, d) == B.CF_EINVAL
    d, keep = _desc(w)
    keep[2][0, B.PARAM_OFFSETS["mass"][0]] = 0.0
    assert _create(lib, d) == B.CF_EINVAL
    d, keep = _desc(w)
    keep[2][1, 40] = np.inf
    assert _create(lib, d) == B.CF_EINVAL
    d, keep = _desc(w, params=None)
    assert _create(lib, d) == B.CF_EINVAL
    # drag and propeller inertia are accepted; a negative propeller inertia is not
    import torch
    ok = B.CF_OK if torch.cuda.is_available() else B.CF_ENODEV
    d, keep = _desc(w)
    keep[2][0, B.PARAM_OFFSETS["drag"][0]] = -0.01
    assert _create(lib, d) == ok
    d, keep = _desc(w)
    fp = int(np.nonzero(w.model_per_world == 0)[0][0])
    keep[2][fp, B.PARAM_OFFSETS["Jp"][0]] = 1e-9
    assert _create(lib, d) == ok
    d, keep = _desc(w)
    keep[2][fp, B.PARAM_OFFSETS["Jp"][0]] = -1e-9
    assert _create(lib, d) == B.CF_EINVAL


def test_create_rejects_out_of_range_gain_index(lib):
    w = W.small("id_rollout_grad", 1)
    gi = np.zeros(w.n_worlds, np.int32)
    gi[5] = 2
    d, keep = _desc(w, n_gains=2, gain_index=gi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert _create(lib, d) == B.CF_EINVAL


def test_create_too_many_drones(lib):
    w = W.small("id_swarm", 1)
    counts = np.full(w.n_worlds, 2 ** 30, np.int32)
    d, keep = _desc(w, drones_per_world=counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert _create(lib, d) == B.CF_EINVAL


def test_valid_create_reports_no_device_or_succeeds(lib):
    d, keep = _desc(W.small("fp_rotor_open_loop", 1))
    st = _create(lib, d)
    import torch
    assert st == (B.CF_OK if torch.cuda.is_available() else B.CF_ENODEV)


def test_null_handle_and_out_arguments(lib):
    assert lib.cf_create(None, None) == B.CF_EINVAL
    assert lib.cf_destroy(None) == B.CF_OK
    assert lib.cf_step_k(None, None, None, 1, None) == B.CF_EINVAL
    assert lib.cf_reset(None, None, None, None) == B.CF_EINVAL
    assert lib.cf_rollout(None, None, None, 1, None, 1, None, None, None, None, None) == B.CF_EINVAL
    assert lib.cf_rollout_backward(None, None, None, 1, None, 1, None, None, None, None, None) == B.CF_EINVAL
    assert lib.cf_autotune(None, None, None, 1, 1) == B.CF_EINVAL
    assert lib.cf_last_error(None) == B.CF_EINVAL
    for code in range(-6, 1):
        assert lib.cf_strerror(code)
    assert lib.cf_strerror(-99) == b"unknown status"


def test_sim_raises_cferror_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("device present")
    with pytest.raises(B.CfError) as ei:
        B.Sim.from_workload(W.small("fp_pid_closed_loop", 1))
    assert ei.value.status == B.CF_ENODEV


def test_torque_interface_descriptor(lib):
    """The torque interface is accepted (it reaches device selection) and, like the
    attitude controller, needs a thrust curve with a positive quadratic term."""
    import torch
    ok = B.CF_OK if torch.cuda.is_available() else B.CF_ENODEV
    w = W.fp_torque(seed=3, n_worlds=8)
    d, keep = _desc(w)
    assert _create(lib, d) == ok
    d, keep = _desc(w)
    keep[2][2, B.PARAM_OFFSETS["thrust_poly"][0] + 2] = 0.0
    assert _create(lib, d) == B.CF_EINVAL


def test_struct_layouts_match_header(tmp_path):
    """Size and field offsets of every C struct of the header, as the host C
    compiler lays them out, equal those of the ctypes mirrors in the binding."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"cf_desc": B._Desc, "cf_objective": B._Objective, "cf_mppi_desc": B._MppiDesc}
    c_name = {"lambda_": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cfsim.h"', "int main(void) {"]
    for s, py in structs.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {c_name.get(f, f)}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for s, py in structs.items():
        assert got[(s, "size")] == ctypes.sizeof(py), s
        for f, _ in py._fields_:
            assert got[(s, f)] == getattr(py, f).offset, (s, f)
