"""Pins of the FP64 oracle against what mathematics fixes independently of it:
closed forms, conservation laws, convergence orders, SciPy's rotation routines,
symmetries, and central finite differences for its gradients.

Each test names the part of the oracle a plausible mistake would break.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

import workloads as W
import oracle as O

F64 = torch.float64


def fp_batch(n=1, control=O.CTRL_ROTOR, integrator=O.RK4, dt=0.002, renorm=1, edit=None):
    P = W.empty_params(n)
    W.fill_fp_airframe(P, np.arange(n), np.full(n, W.MASS), np.tile(W.INERTIA, (n, 1)))
    if edit:
        edit(P)
    return O.Batch(np.ones(n, np.int64), np.zeros(n), P, control, integrator, dt, renorm), P


def id_batch(n=1, integrator=O.RK4, dt=0.002, gain=None, tau=None, edit=None):
    P = W.empty_params(n)
    W.fill_id_model(P, np.arange(n), np.tile(W.ID_GAIN if gain is None else gain, (n, 1)),
                    np.tile(W.ID_TAU if tau is None else tau, (n, 1)))
    if edit:
        edit(P)
    return O.Batch(np.ones(n, np.int64), np.ones(n), P, O.CTRL_ATT_PID, integrator, dt), P


def run(b, x, u, n):
    with torch.no_grad():
        for _ in range(n):
            x = b.step(x, u)
    return x


def unit_quats(rng, n):
    q = rng.normal(size=(4, n))
    return q / np.linalg.norm(q, axis=0)


# ---- gravity, translation, integrator plumbing -------------------------------------

@pytest.mark.parametrize("integ", [O.RK4, O.EULER])
def test_free_fall_first_principles(integ):
    """Zero rotor speed and command, k0 = 0: no thrust, only gravity. RK4 is exact
    on the quadratic; explicit Euler has the closed-form lag g t dt / 2."""
    rng = np.random.default_rng(0)
    dt, n = 0.002, 400
    b, _ = fp_batch(3, integrator=integ, dt=dt)
    x = torch.zeros(17, 3, dtype=F64)
    x[0:3] = torch.as_tensor(rng.uniform(-1, 1, (3, 3)))
    x[3:7] = torch.as_tensor(unit_quats(rng, 3))
    x[7:10] = torch.as_tensor(rng.normal(0, 1, (3, 3)))
    y = run(b, x, torch.zeros(4, 3, dtype=F64), n)
    t = n * dt
    expect = x[0:3] + x[7:10] * t
    expect[2] -= 0.5 * W.GRAVITY * t * t
    if integ == O.EULER:
        expect[2] += 0.5 * W.GRAVITY * t * dt
    assert torch.allclose(y[0:3], expect, rtol=0, atol=1e-12)
    assert torch.allclose(y[7:10], x[7:10] - torch.tensor([0, 0, W.GRAVITY * t], dtype=F64)[:, None], atol=1e-12)


@pytest.mark.parametrize("integ", [O.RK4, O.EULER])
def test_free_fall_identified(integ):
    dt, n = 0.002, 300
    b, _ = id_batch(2, integrator=integ, dt=dt)
    x = torch.zeros(13, 2, dtype=F64)
    x[3:6] = torch.tensor([[0.1, -0.2], [0.05, 0.1], [0.3, -0.4]], dtype=F64)
    x[6:9] = torch.tensor([[1.0, 0.0], [0.0, -2.0], [0.5, 0.0]], dtype=F64)
    u = torch.zeros(4, 2, dtype=F64)
    y = run(b, x, u, n)
    t = n * dt
    expect = x[0:3] + x[6:9] * t
    expect[2] -= 0.5 * W.GRAVITY * t * t
    if integ == O.EULER:
        expect[2] += 0.5 * W.GRAVITY * t * dt
    assert torch.allclose(y[0:3], expect, atol=1e-12)


# ---- hover: thrust curve, mixing symmetry, gravity sign -------------------------------

def test_hover_first_principles_rotor():
    b, P = fp_batch(2)
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(17, 2, dtype=F64)
    x[0:3] = torch.tensor([[0.3, -1.0], [0.2, 0.0], [1.0, 2.0]], dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    y = run(b, x, torch.full((4, 2), wh, dtype=F64), 1000)
    assert torch.allclose(y, x, rtol=0, atol=1e-9 * wh)
    assert torch.allclose(y[0:13], x[0:13], rtol=0, atol=1e-12)


def test_hover_first_principles_pid():
    """Zero attitude error and thrust command m g: integrators stay at zero, every
    rotor is commanded the hover speed and the state does not move."""
    b, P = fp_batch(2, control=O.CTRL_ATT_PID)
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(25, 2, dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    u = torch.tensor([[0.0] * 2, [0.0] * 2, [0.0] * 2, [W.MASS * W.GRAVITY] * 2], dtype=F64)
    y = run(b, x, u, 1000)
    assert torch.allclose(y[0:13], x[0:13], atol=1e-11)
    assert torch.allclose(y[13:17], x[13:17], rtol=1e-12)
    assert torch.allclose(y[17:25], x[17:25], atol=1e-12)


def test_hover_identified():
    b, P = id_batch(2)
    fh = W.MASS * W.GRAVITY / W.ID_CF
    x = torch.zeros(13, 2, dtype=F64)
    x[12] = fh
    u = torch.tensor([[0.0] * 2] * 3 + [[fh] * 2], dtype=F64)
    y = run(b, x, u, 1000)
    assert torch.allclose(y, x, atol=1e-12)


# ---- rotor dynamics --------------------------------------------------------------------

@pytest.mark.parametrize("integ", [O.RK4, O.EULER])
def test_rotor_discrete_closed_form_both_branches(integ):
    """Linear rotor law: Omega_n - Omega_c = (Omega_0 - Omega_c) P(c dt)^n with
    P(z) = 1 - z + z^2/2 - z^3/6 + z^4/24 (RK4) or 1 - z (Euler). Distinct
    acceleration and deceleration coefficients pin the branch selection."""
    cv_up, cv_dn, dt, n = 40.0, 15.0, 0.002, 200

    def edit(P):
        P["motor_up"][:] = (cv_up, 0.0)
        P["motor_down"][:] = (cv_dn, 0.0)

    b, _ = fp_batch(1, integrator=integ, dt=dt, edit=edit)
    x = torch.zeros(17, 1, dtype=F64)
    x[6] = 1.0
    x[13:17, 0] = torch.tensor([10000.0, 20000.0, 12000.0, 18000.0], dtype=F64)
    cmd = torch.tensor([[15000.0], [15000.0], [16000.0], [16000.0]], dtype=F64)
    y = run(b, x, cmd, n)

    def amp(z):
        return 1 - z + z * z / 2 - z ** 3 / 6 + z ** 4 / 24 if integ == O.RK4 else 1 - z

    for i in range(4):
        c = cv_up if cmd[i, 0] >= x[13 + i, 0] else cv_dn
        expect = cmd[i, 0] + (x[13 + i, 0] - cmd[i, 0]) * amp(c * dt) ** n
        assert abs(float(y[13 + i, 0] - expect)) < 1e-9


def test_rotor_quadratic_bernoulli():
    """With c_d != 0 the error e = Omega_c - Omega obeys the Bernoulli equation
    e' = -a e + c_d e^2 (a = c_v + 2 c_d Omega_c), solved in closed form; RK4
    converges to it at fourth order."""
    cv, cd = 20.0, 2e-3
    wc, w0, T = 15000.0, 9000.0, 0.1

    def edit(P):
        P["motor_up"][:] = (cv, cd)
        P["motor_down"][:] = (cv, cd)

    a = cv + 2 * cd * wc
    e0 = wc - w0
    e_exact = a * e0 * math.exp(-a * T) / (a - cd * e0 * (1 - math.exp(-a * T)))
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        b, _ = fp_batch(1, dt=dt, edit=edit)
        x = torch.zeros(17, 1, dtype=F64)
        x[6] = 1.0
        x[13:17] = w0
        y = run(b, x, torch.full((4, 1), wc, dtype=F64), int(round(T / dt)))
        errs.append(abs(float(wc - y[13, 0]) - e_exact))
    assert errs[0] < 1e-2 * e0 * 1e-3
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


# ---- quaternion kinematics ---------------------------------------------------------------

def _spin_batch(integ, dt, renorm):
    def edit(P):
        P["J"][:] = (2e-5, 2e-5, 2e-5)       # isotropic: w x J w = 0, w stays constant
    return fp_batch(1, integrator=integ, dt=dt, renorm=renorm, edit=edit)[0]


@pytest.mark.parametrize("integ", [O.RK4, O.EULER])
def test_quaternion_norm_closed_form_without_renormalisation(integ):
    """For constant w, q' = 1/2 q (x) [w,0] is linear with a skew generator; the
    RK4 map scales |q|^2 by 1 - th^6/72 + th^8/576 per step, Euler by 1 + th^2,
    th = |w| dt / 2."""
    dt, n = 0.01, 100
    w = np.array([20.0, -10.0, 25.0])
    b = _spin_batch(integ, dt, renorm=0)
    x = torch.zeros(17, 1, dtype=F64)
    x[3:7, 0] = torch.as_tensor(unit_quats(np.random.default_rng(1), 1)[:, 0])
    x[10:13, 0] = torch.as_tensor(w)
    y = run(b, x, torch.zeros(4, 1, dtype=F64), n)
    th = np.linalg.norm(w) * dt / 2
    fac = (1 - th ** 6 / 72 + th ** 8 / 576) if integ == O.RK4 else (1 + th * th)
    assert abs(float((y[3:7, 0] ** 2).sum()) - fac ** n) < 1e-12 * fac ** n


def test_quaternion_constant_rate_matches_scipy():
    """With renormalisation, integrating body rate w from q0 gives
    q0 (x) exp(w t / 2) -- right multiplication, scalar last -- compared with
    SciPy's Rotation composition; also checks |q| = 1."""
    dt, n = 0.002, 500
    rng = np.random.default_rng(2)
    b = _spin_batch(O.RK4, dt, renorm=1)
    for _ in range(3):
        q0 = unit_quats(rng, 1)[:, 0]
        w = rng.normal(0, 3, 3)
        x = torch.zeros(17, 1, dtype=F64)
        x[3:7, 0] = torch.as_tensor(q0)
        x[10:13, 0] = torch.as_tensor(w)
        y = run(b, x, torch.zeros(4, 1, dtype=F64), n)[3:7, 0].numpy()
        ref = (Rotation.from_quat(q0) * Rotation.from_rotvec(w * n * dt)).as_quat()
        if np.dot(ref, y) < 0:
            ref = -ref
        assert np.abs(y - ref).max() < 1e-10
        assert abs(np.linalg.norm(y) - 1) < 1e-14


def test_rotation_helpers_match_scipy():
    rng = np.random.default_rng(3)
    q = unit_quats(rng, 50)
    Rz = Rotation.from_quat(q.T).apply([0.0, 0.0, 1.0]).T
    assert np.allclose(O.body_z_in_world(torch.as_tensor(q)).numpy(), Rz, atol=1e-14)
    roll, pitch = O.roll_pitch_from_quat(torch.as_tensor(q))
    eul = Rotation.from_quat(q.T).as_euler("ZYX")         # yaw, pitch, roll
    assert np.allclose(roll.numpy(), eul[:, 2], atol=1e-12)
    assert np.allclose(pitch.numpy(), eul[:, 1], atol=1e-12)
    psi = rng.uniform(-1, 1, (3, 50))
    Rp = Rotation.from_euler("ZYX", psi[::-1].T).apply([0.0, 0.0, 1.0]).T
    assert np.allclose(O.euler_zyx_body_z(torch.as_tensor(psi)).numpy(), Rp, atol=1e-14)
    a, bq = unit_quats(rng, 20), unit_quats(rng, 20)
    ref = (Rotation.from_quat(a.T) * Rotation.from_quat(bq.T)).as_quat().T
    got = O.quat_mul(torch.as_tensor(a), torch.as_tensor(bq)).numpy()
    sign = np.sign((ref * got).sum(0))
    assert np.allclose(got, ref * sign, atol=1e-14)


# ---- Euler's rigid-body equations ------------------------------------------------------------

def test_torque_free_axisymmetric_precession():
    """J_x = J_y: w_z constant and (w_x + i w_y) rotates at (J_z - J_x) w_z / J_x;
    the RK4 phase error against that closed form shrinks at fourth order."""
    Jx, Jz = W.INERTIA[0], W.INERTIA[2]
    w0 = np.array([3.0, -2.0, 40.0])
    lam = (Jz - Jx) * w0[2] / Jx
    errs = []
    for dt in (2e-3, 1e-3):
        n = int(round(1.0 / dt))
        b, P = fp_batch(1, dt=dt)
        x = torch.zeros(17, 1, dtype=F64)
        x[6] = 1.0
        x[10:13, 0] = torch.as_tensor(w0)
        y = run(b, x, torch.zeros(4, 1, dtype=F64), n)[10:13, 0].numpy()
        c = (w0[0] + 1j * w0[1]) * np.exp(1j * lam * n * dt)
        assert abs(y[2] - w0[2]) < 1e-12
        errs.append(abs(complex(y[0], y[1]) - c))
    assert errs[1] < 1e-6
    assert 13 < errs[0] / errs[1] < 19, errs


def test_torque_free_triaxial_conservation():
    """Triaxial J: kinetic energy, |J w| and the world-frame angular momentum
    R(q) J w are invariants; their RK4 drift shrinks at fourth order."""
    def edit(P):
        P["J"][:] = (1.3e-5, 1.55e-5, 2.3e-5)
    J = np.array([1.3e-5, 1.55e-5, 2.3e-5])
    w0 = np.array([8.0, -12.0, 5.0])
    q0 = unit_quats(np.random.default_rng(4), 1)[:, 0]
    drifts = []
    for dt in (4e-3, 2e-3):
        b, _ = fp_batch(1, dt=dt, edit=edit)
        x = torch.zeros(17, 1, dtype=F64)
        x[3:7, 0] = torch.as_tensor(q0)
        x[10:13, 0] = torch.as_tensor(w0)
        y = run(b, x, torch.zeros(4, 1, dtype=F64), int(round(1.0 / dt)))
        w, q = y[10:13, 0].numpy(), y[3:7, 0].numpy()
        E0, E = 0.5 * (J * w0 * w0).sum(), 0.5 * (J * w * w).sum()
        L0 = Rotation.from_quat(q0).apply(J * w0)
        L = Rotation.from_quat(q).apply(J * w)
        assert abs(E - E0) < 1e-6 * E0
        assert abs(np.linalg.norm(J * w) - np.linalg.norm(J * w0)) < 1e-6 * np.linalg.norm(J * w0)
        assert np.abs(L - L0).max() < 1e-6 * np.linalg.norm(L0)
        drifts.append(np.abs(L - L0).max())
    assert 10 < drifts[0] / drifts[1] < 24


# ---- integrator order ------------------------------------------------------------------------

@pytest.mark.parametrize("integ,ratio", [(O.RK4, 16.0), (O.EULER, 2.0)])
def test_convergence_order(integ, ratio):
    """Held rotor commands above the initial speeds (no branch change), tilted
    and spinning: error at T against a dt/64 RK4 reference halves like dt^order."""
    T, dt0 = 0.2, 4e-3
    x = torch.zeros(17, 1, dtype=F64)
    x[3:7, 0] = torch.tensor([0.1, -0.2, 0.05, 0.97], dtype=F64) / math.sqrt(0.01 + 0.04 + 0.0025 + 0.97 ** 2)
    x[7:10, 0] = torch.tensor([0.5, -0.3, 0.2], dtype=F64)
    x[10:13, 0] = torch.tensor([2.0, -1.0, 3.0], dtype=F64)
    x[13:17, 0] = torch.tensor([13000.0, 14000.0, 13500.0, 14200.0], dtype=F64)
    cmd = torch.tensor([[15500.0], [15000.0], [16000.0], [15200.0]], dtype=F64)
    bref, _ = fp_batch(1, integrator=O.RK4, dt=dt0 / 64)
    ref = run(bref, x, cmd, int(round(T / (dt0 / 64))))
    errs = []
    for k in range(3):
        dt = dt0 / 2 ** k
        b, _ = fp_batch(1, integrator=integ, dt=dt)
        y = run(b, x, cmd, int(round(T / dt)))
        errs.append(float((y[0:13] - ref[0:13]).abs().max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 0.75 * ratio < r1 < 1.3 * ratio and 0.75 * ratio < r2 < 1.3 * ratio, errs


# ---- identified model -----------------------------------------------------------------------

def test_identified_attitude_lti_discrete_closed_form():
    """Per axis z = [Psi, Psi'] obeys z' = A z + b Psi_c with A = [[0,1],[c1,c2]];
    RK4 on an affine system is exactly z+ = R(hA) z + h S(hA) b Psi_c with
    R(X) = I+X+X^2/2+X^3/6+X^4/24, S(X) = I+X/2+X^2/6+X^3/24. The thrust state
    follows f_c + (f0 - f_c) P(c_tau dt)^n; the continuous solution (matrix
    exponential) is approached at O(dt^4); steady state is k Psi_c."""
    dt, n = 0.002, 400
    gain, tau = np.array([1.1, 0.9, 1.2]), np.array([0.07, 0.05, 0.11])
    b, P = id_batch(1, dt=dt, gain=gain, tau=tau)
    x = torch.zeros(13, 1, dtype=F64)
    x[3:6, 0] = torch.tensor([0.05, -0.1, 0.2], dtype=F64)
    x[9:12, 0] = torch.tensor([0.3, 0.0, -0.5], dtype=F64)
    x[12, 0] = 0.2
    u = torch.tensor([[0.15], [-0.05], [0.4], [0.3]], dtype=F64)
    y = run(b, x, u, n)
    I2 = np.eye(2)
    for ax in range(3):
        c1, c2, c3 = P["c_psi1"][0, ax], P["c_psi2"][0, ax], P["c_psi3"][0, ax]
        A = np.array([[0.0, 1.0], [c1, c2]])
        X = dt * A
        R = I2 + X + X @ X / 2 + X @ X @ X / 6 + X @ X @ X @ X / 24
        S = I2 + X / 2 + X @ X / 6 + X @ X @ X / 24
        bvec = np.array([0.0, c3 * float(u[ax, 0])])
        z = np.array([float(x[3 + ax, 0]), float(x[9 + ax, 0])])
        for _ in range(n):
            z = R @ z + dt * S @ bvec
        assert abs(z[0] - float(y[3 + ax, 0])) < 1e-12 and abs(z[1] - float(y[9 + ax, 0])) < 1e-11
        # continuous solution (augmented matrix exponential)
        Aug = np.zeros((3, 3))
        Aug[0:2, 0:2] = A
        Aug[0:2, 2] = bvec
        zc = (expm(Aug * n * dt) @ np.array([float(x[3 + ax, 0]), float(x[9 + ax, 0]), 1.0]))[0:2]
        assert abs(zc[0] - z[0]) < 1e-7
    ct = P["c_tau"][0, 0]
    zt = ct * dt
    amp = 1 - zt + zt ** 2 / 2 - zt ** 3 / 6 + zt ** 4 / 24
    assert abs(float(y[12, 0]) - (0.3 + (0.2 - 0.3) * amp ** n)) < 1e-12
    # steady state: Psi -> k Psi_c
    y2 = run(b, x, u, 5000)
    assert np.allclose(y2[3:6, 0].numpy(), gain * u[0:3, 0].numpy(), atol=1e-9)


# ---- symmetries --------------------------------------------------------------------------

def _yaw_quat(beta):
    return torch.tensor([0.0, 0.0, math.sin(beta / 2), math.cos(beta / 2)], dtype=F64)


def _rotz(beta):
    c, s = math.cos(beta), math.sin(beta)
    return torch.tensor([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=F64)


@pytest.mark.parametrize("control", [O.CTRL_ROTOR, O.CTRL_ATT_PID])
def test_yaw_equivariance_first_principles(control):
    """Rotating the initial position, velocity and attitude about world z rotates
    the whole trajectory (gravity is along z; body quantities are unchanged)."""
    rng = np.random.default_rng(5)
    beta = 0.7
    S = 25 if control == O.CTRL_ATT_PID else 17
    b, _ = fp_batch(2, control=control)
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(S, 2, dtype=F64)
    x[0:3] = torch.as_tensor(rng.normal(size=(3, 2)))
    x[3:7] = torch.as_tensor(unit_quats(rng, 2))
    x[7:10] = torch.as_tensor(rng.normal(size=(3, 2)))
    x[10:13] = torch.as_tensor(rng.normal(0, 0.5, size=(3, 2)))
    x[13:17] = wh
    if control == O.CTRL_ATT_PID:
        x[22:25] = x[10:13]
        u = torch.tensor([[0.1, -0.2], [0.05, 0.2], [0.3, -0.1], [0.3, 0.25]], dtype=F64)
    else:
        u = torch.as_tensor(wh * (1 + 0.05 * rng.normal(size=(4, 2))))
    Rz = _rotz(beta)
    xr = x.clone()
    xr[0:3] = Rz @ x[0:3]
    xr[7:10] = Rz @ x[7:10]
    xr[3:7] = O.quat_mul(_yaw_quat(beta)[:, None].expand(4, 2), x[3:7])
    y = run(b, x, u, 300)
    yr = run(b, xr, u, 300)
    assert torch.allclose(yr[0:3], Rz @ y[0:3], atol=1e-10)
    assert torch.allclose(yr[7:10], Rz @ y[7:10], atol=1e-10)
    assert torch.allclose(yr[10:], y[10:], atol=1e-9 * wh)
    qy = O.quat_mul(_yaw_quat(beta)[:, None].expand(4, 2), y[3:7])
    assert torch.allclose(yr[3:7], qy, atol=1e-10)


def test_yaw_equivariance_and_translation_identified():
    b, _ = id_batch(1)
    beta = -0.9
    x = torch.zeros(13, 1, dtype=F64)
    x[0:3, 0] = torch.tensor([1.0, 2.0, 3.0], dtype=F64)
    x[3:6, 0] = torch.tensor([0.1, -0.05, 0.3], dtype=F64)
    x[6:9, 0] = torch.tensor([0.5, -1.0, 0.2], dtype=F64)
    x[12, 0] = 0.3
    u = torch.tensor([[0.05], [0.1], [0.2], [0.28]], dtype=F64)
    y = run(b, x, u, 400)
    xr, ur = x.clone(), u.clone()
    xr[0:3] = _rotz(beta) @ x[0:3] + torch.tensor([[5.0], [-3.0], [1.0]], dtype=F64)
    xr[6:9] = _rotz(beta) @ x[6:9]
    xr[5] += beta
    ur[2] += beta          # yaw is commanded as an absolute angle (DC gain 1 here)
    yr = run(b, xr, ur, 400)
    assert torch.allclose(yr[0:3], _rotz(beta) @ y[0:3] + torch.tensor([[5.0], [-3.0], [1.0]], dtype=F64), atol=1e-10)
    assert torch.allclose(yr[6:9], _rotz(beta) @ y[6:9], atol=1e-10)


# ---- mixing and controller -------------------------------------------------------------------

def test_single_rotor_torque_matches_cross_product():
    """Torque of one rotor's thrust equals r_i x (f e_z) for the x-airframe motor
    positions M1(+a,-a) M2(-a,-a) M3(-a,+a) M4(+a,+a); the reaction torque about
    z follows the spin signs -,+,-,+ at the torque/thrust ratio."""
    _, P = fp_batch(1)
    Pd = O.per_drone_params(P, [1])
    a = W.ARM / math.sqrt(2)
    pos = np.array([[a, -a, 0], [-a, -a, 0], [-a, a, 0], [a, a, 0]])
    for i in range(4):
        rot = torch.zeros(4, 1, dtype=F64)
        rot[i] = 15000.0
        thrust, torque = O.rotor_wrench(rot, Pd)
        f = W.K_THRUST * 15000.0 ** 2
        assert abs(float(thrust[0]) - f) < 1e-15
        expect = np.cross(pos[i], [0, 0, f])
        assert np.allclose(torque[0:2, 0].numpy(), expect[0:2], atol=1e-18)
        assert abs(float(torque[2, 0]) - (-1) ** (i + 1) * W.TORQUE_RATIO * f) < 1e-18


def test_allocation_inverts_mixing():
    _, P = fp_batch(1)
    a = W.ARM / math.sqrt(2)
    mix = np.stack([np.ones(4), P["mix_tx"][0], P["mix_ty"][0], W.TORQUE_RATIO * P["mix_yaw"][0]])
    assert np.allclose(P["alloc"][0].reshape(4, 4) @ mix, np.eye(4), atol=1e-12)
    assert np.allclose(mix[1], a * np.array([-1, -1, 1, 1]))


def test_pid_closed_loop_linearisation_is_stable():
    """Jacobian of the closed-loop discrete map at hover: every mode that the loop
    controls lies strictly inside the unit circle; the only unit modes are the
    uncontrolled ones (position 3, velocity 3, yaw angle 1)."""
    b, _ = fp_batch(1, control=O.CTRL_ATT_PID)
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(25, 1, dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    u = torch.tensor([[0.0], [0.0], [0.0], [W.MASS * W.GRAVITY]], dtype=F64)
    scale = torch.ones(25, dtype=F64)
    scale[13:17] = wh
    Jm = torch.zeros(25, 25, dtype=F64)
    for j in range(25):
        h = 1e-6 * scale[j]
        xp, xm = x.clone(), x.clone()
        xp[j] += h
        xm[j] -= h
        Jm[:, j] = (b.step(xp, u) - b.step(xm, u))[:, 0] / (2 * h)
    # quaternion: drop w (renormalisation removes the radial direction)
    keep = [i for i in range(25) if i != 6]
    ev = np.linalg.eigvals(Jm[keep][:, keep].numpy())
    mag = np.sort(np.abs(ev))[::-1]
    assert mag[0] < 1 + 1e-7
    assert np.sum(mag > 1 - 1e-7) == 7
    assert mag[7] < 1 - 1e-5


def test_pid_tracks_held_attitude():
    b, _ = fp_batch(1, control=O.CTRL_ATT_PID)
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(25, 1, dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    u = torch.tensor([[0.2], [-0.1], [0.3], [W.MASS * W.GRAVITY]], dtype=F64)
    y = run(b, x, u, 15000)
    roll, pitch = O.roll_pitch_from_quat(y[3:7])
    assert abs(float(roll[0]) - 0.2) < 2e-3 and abs(float(pitch[0]) + 0.1) < 2e-3
    assert abs(float(y[12, 0]) - 0.3) < 2e-3


# ---- gradients -------------------------------------------------------------------------------

def _fd_check(w, n_dirs=4, h=1e-4, seed=0):
    """Central differences of the FP64 oracle loss along random directions of the
    per-step commands, the initial state and the gain vs the autograd gradient."""
    b = O.Batch.from_workload(w)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u,
              ref_offset=None if w.ref_offset is None else O.t64(w.ref_offset), reward=w.reward,
              policy_hidden=w.policy_hidden)
    x0, cmds = O.t64(w.x0), O.t64(w.cmds)
    gain = None if w.gain is None else O.t64(w.gain)
    g = O.rollout_grad(b, x0, cmds, w.steps, gain=gain, gain_index=w.gain_index, dloss=w.dloss, **kw)
    seed_w = O.t64(w.dloss)

    def L(x0_, c_, g_):
        with torch.no_grad():
            out = O.rollout(b, x0_, c_, w.steps, gain=g_, gain_index=w.gain_index, **kw)
        return float((seed_w * out["loss"]).sum())

    rng = np.random.default_rng(seed)
    scale_x = torch.ones_like(x0)
    if x0.shape[0] >= 17:
        scale_x[13:17] = 1e3
    for _ in range(n_dirs):
        dx = torch.as_tensor(rng.normal(size=x0.shape)) * scale_x
        if x0.shape[0] >= 17:
            dx[3:7] = 0          # keep the attitude direction out (renormalised)
        dc = torch.as_tensor(rng.normal(size=cmds.shape))
        if x0.shape[0] >= 17 and w.control == O.CTRL_ROTOR:
            dc *= 1e3
        dg = None if gain is None else torch.as_tensor(rng.normal(size=gain.shape))
        fp = L(x0 + h * dx, cmds + h * dc, None if gain is None else gain + h * dg)
        fm = L(x0 - h * dx, cmds - h * dc, None if gain is None else gain - h * dg)
        fd = (fp - fm) / (2 * h)
        ad = float((g["g_x0"] * dx).sum() + (g["g_cmds"] * dc).sum())
        if gain is not None:
            ad += float((g["g_gain"] * dg).sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3), (fd, ad)
    return g


def test_gradient_fd_identified_with_feedback():
    w = W.id_rollout_grad(seed=11, n_worlds=3, steps=40, gain_std=0.05)
    _fd_check(w)


def test_gradient_fd_first_principles_pid():
    w = W.uneven_mixed_adjoint(seed=12, n_worlds=6, n_subset=4, steps=30, n_max=3)
    _fd_check(w)


def test_gradient_fd_first_principles_rotor():
    w = W.fp_rotor_open_loop(seed=13, n_worlds=2, steps=30)
    w.ref_offset = w.x0[0:3].copy()
    w.dloss = np.ones(2, np.float32)
    w.w_u = 1e-9
    _fd_check(w, h=1e-3)


def test_gradient_fd_asymmetric_rotor_law_away_from_the_kink():
    """Distinct acceleration/deceleration coefficients with quadratic terms:
    commands held 20 % above or below hover per rotor, so no rotor's command
    crosses its speed in 20 steps (no branch switch) and the central
    differences see a smooth map."""
    w = W.fp_rotor_open_loop(seed=15, n_worlds=3, steps=20)
    w.params["motor_up"][:] = (40.0, 5e-4)
    w.params["motor_down"][:] = (20.0, 1e-3)
    hov = float(W.hover_speed(W.MASS))
    sgn = np.array([[1.0, -1.0, 1.0], [-1.0, -1.0, 1.0], [1.0, 1.0, -1.0], [-1.0, 1.0, 1.0]])
    w.cmds = np.broadcast_to(hov * (1.0 + 0.2 * sgn), (w.steps, 4, 3)).astype(np.float32).copy()
    w.ref_offset = w.x0[0:3].copy()
    w.dloss = np.ones(3, np.float32)
    w.w_u = 1e-9
    _fd_check(w, h=1e-3)


def test_gain_gradient_identity():
    """u_t = ubar_t + G e_t gives dL/dG = sum_t (dL/du_t) e_t^T exactly."""
    w = W.id_rollout_grad(seed=14, n_worlds=4, steps=25, gain_std=0.05)
    b = O.Batch.from_workload(w)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    g = O.rollout_grad(b, w.x0, w.cmds, w.steps, gain=O.t64(w.gain), dloss=w.dloss, **kw)
    out = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, gain=O.t64(w.gain), keep_traj=True, **kw)
    traj = out["traj"].detach()
    acc = torch.zeros(4, 13, dtype=F64)
    for n in range(w.steps):
        p, v = b.figure_eight(n * b.dt, w.ref_amp, w.ref_period, None)
        e = traj[n, 0:13] - b.reference_state(p, v)
        acc += g["g_cmds"][n] @ e.T
    assert torch.allclose(acc, g["g_gain"][0], rtol=1e-10, atol=1e-14)


# ---- rotor gyroscopic/reaction torques and linear drag ----------------------------------------

def test_rotation_matrices_match_scipy():
    rng = np.random.default_rng(20)
    q = unit_quats(rng, 30)
    assert np.allclose(O.rotation_matrix(torch.as_tensor(q)).numpy().transpose(2, 0, 1),
                       Rotation.from_quat(q.T).as_matrix(), atol=1e-14)
    psi = rng.uniform(-1, 1, (3, 30))
    assert np.allclose(O.euler_zyx_matrix(torch.as_tensor(psi)).numpy().transpose(2, 0, 1),
                       Rotation.from_euler("ZYX", psi[::-1].T).as_matrix(), atol=1e-14)


def _gyro_batch(dt, jp=4e-9):
    def edit(P):
        P["Jp"][:] = jp
        P["torque_poly"][:] = 0.0          # no rotor drag torque: no external torque at all
        P["J"][:] = (1.3e-5, 1.55e-5, 2.3e-5)
    return fp_batch(1, dt=dt, edit=edit)


def test_gyroscopic_total_angular_momentum_conserved():
    """Rotors at steady speeds (a, b, a, b): thrust and yaw torques vanish, so the
    total angular momentum R(q) (J w + J_p Omega_s e_z) is conserved; the RK4
    drift shrinks at fourth order. A wrong sign of the gyroscopic rows breaks
    conservation at first order."""
    J = np.array([1.3e-5, 1.55e-5, 2.3e-5])
    jp = 4e-9
    speeds = np.array([18000.0, 9000.0, 18000.0, 9000.0])
    om_s = speeds[0] - speeds[1] + speeds[2] - speeds[3]
    q0 = unit_quats(np.random.default_rng(21), 1)[:, 0]
    w0 = np.array([6.0, -9.0, 4.0])
    drifts = []
    for dt in (2e-3, 1e-3):
        b, _ = _gyro_batch(dt, jp)
        x = torch.zeros(17, 1, dtype=F64)
        x[3:7, 0] = torch.as_tensor(q0)
        x[10:13, 0] = torch.as_tensor(w0)
        x[13:17, 0] = torch.as_tensor(speeds)
        y = run(b, x, torch.as_tensor(speeds[:, None]), int(round(0.5 / dt)))
        w, q = y[10:13, 0].numpy(), y[3:7, 0].numpy()
        L0 = Rotation.from_quat(q0).apply(J * w0 + np.array([0, 0, jp * om_s]))
        L = Rotation.from_quat(q).apply(J * w + np.array([0, 0, jp * om_s]))
        drifts.append(np.abs(L - L0).max())
        assert drifts[-1] < 1e-6 * np.linalg.norm(L0)
    assert 10 < drifts[0] / drifts[1] < 24
    # the gyroscopic term matters here: without it the momentum is not conserved
    b, _ = _gyro_batch(1e-3, 0.0)
    x = torch.zeros(17, 1, dtype=F64)
    x[3:7, 0] = torch.as_tensor(q0)
    x[10:13, 0] = torch.as_tensor(w0)
    x[13:17, 0] = torch.as_tensor(speeds)
    y = run(b, x, torch.as_tensor(speeds[:, None]), 500)
    L = Rotation.from_quat(y[3:7, 0].numpy()).apply(J * y[10:13, 0].numpy() + np.array([0, 0, jp * om_s]))
    assert np.abs(L - L0).max() > 1e3 * drifts[1]


def test_reaction_torque_of_rotor_spin_up():
    """Spinning up rotors 1 and 3 from rest with no external torque: the body yaws
    the other way, J_z w_z = -J_p (Omega_1 + Omega_3), exactly (RK4 integrates
    both sides with the same weights)."""
    jp = 4e-9
    b, _ = _gyro_batch(2e-3, jp)
    x = torch.zeros(17, 1, dtype=F64)
    x[6] = 1.0
    cmd = torch.tensor([[16000.0], [0.0], [16000.0], [0.0]], dtype=F64)
    y = run(b, x, cmd, 150)
    om_s = float(y[13, 0] - y[14, 0] + y[15, 0] - y[16, 0])
    assert om_s > 1e4
    assert abs(float(y[12, 0]) * 2.3e-5 + jp * om_s) < 1e-15 * jp * om_s * 1e3
    assert abs(float(y[10, 0])) < 1e-12 and abs(float(y[11, 0])) < 1e-12


def _affine_rk4(A, b, z0, h, n):
    I = np.eye(len(z0))
    X = h * A
    R = I + X + X @ X / 2 + X @ X @ X / 6 + X @ X @ X @ X / 24
    S = I + X / 2 + X @ X / 6 + X @ X @ X / 24
    z = z0.copy()
    for _ in range(n):
        z = R @ z + h * S @ b
    return z


DRAG = np.array([-0.004, -0.006, -0.009])


def test_drag_first_principles_exact_affine_map():
    """Constant attitude, no rotor thrust: [p, v]' = [v, R C_a R^T v / m - g e_z]
    is affine; the RK4 map is R4(hA) z + h S4(hA) b exactly. A transposed
    rotation (R^T C_a R) fails it for a generic attitude."""
    dt, n = 2e-3, 300

    def edit(P):
        P["drag"][:] = DRAG
    b, P = fp_batch(1, dt=dt, edit=edit)
    q0 = unit_quats(np.random.default_rng(22), 1)[:, 0]
    x = torch.zeros(17, 1, dtype=F64)
    x[3:7, 0] = torch.as_tensor(q0)
    x[0:3, 0] = torch.tensor([0.3, -0.2, 1.0], dtype=F64)
    x[7:10, 0] = torch.tensor([2.0, -1.5, 0.7], dtype=F64)
    y = run(b, x, torch.zeros(4, 1, dtype=F64), n)
    Rm = Rotation.from_quat(q0).as_matrix()
    M = Rm @ np.diag(DRAG) @ Rm.T / W.MASS
    A = np.zeros((6, 6))
    A[0:3, 3:6] = np.eye(3)
    A[3:6, 3:6] = M
    bb = np.array([0, 0, 0, 0, 0, -W.GRAVITY])
    z = _affine_rk4(A, bb, np.concatenate([x[0:3, 0].numpy(), x[7:10, 0].numpy()]), dt, n)
    assert np.allclose(y[0:3, 0].numpy(), z[0:3], atol=1e-12)
    assert np.allclose(y[7:10, 0].numpy(), z[3:6], atol=1e-12)
    Mt = Rm.T @ np.diag(DRAG) @ Rm / W.MASS
    A[3:6, 3:6] = Mt
    zt = _affine_rk4(A, bb, np.concatenate([x[0:3, 0].numpy(), x[7:10, 0].numpy()]), dt, n)
    assert np.abs(zt[3:6] - z[3:6]).max() > 1e-3


def test_drag_identified_exact_affine_map():
    dt, n = 2e-3, 300

    def edit(P):
        P["drag"][:] = DRAG
    b, P = id_batch(1, dt=dt, edit=edit)
    psi = np.array([0.2, -0.3, 0.9])
    x = torch.zeros(13, 1, dtype=F64)
    x[3:6, 0] = torch.as_tensor(psi)
    x[6:9, 0] = torch.tensor([1.0, 2.0, -0.5], dtype=F64)
    u = torch.tensor([[psi[0]], [psi[1]], [psi[2]], [0.0]], dtype=F64)   # DC gain 1 holds the attitude
    y = run(b, x, u, n)
    assert np.allclose(y[3:6, 0].numpy(), psi, atol=1e-14)
    Rm = Rotation.from_euler("ZYX", psi[::-1]).as_matrix()
    A = np.zeros((6, 6))
    A[0:3, 3:6] = np.eye(3)
    A[3:6, 3:6] = Rm @ np.diag(DRAG) @ Rm.T / W.MASS
    bb = np.array([0, 0, 0, 0, 0, -W.GRAVITY])
    z = _affine_rk4(A, bb, np.concatenate([x[0:3, 0].numpy(), x[6:9, 0].numpy()]), dt, n)
    assert np.allclose(y[0:3, 0].numpy(), z[0:3], atol=1e-12)
    assert np.allclose(y[6:9, 0].numpy(), z[3:6], atol=1e-12)


def test_gradient_fd_with_gyro_and_drag():
    for w in (W.uneven_mixed_adjoint(seed=23, n_worlds=6, n_subset=4, steps=30, n_max=3),
              W.id_rollout_grad(seed=24, n_worlds=3, steps=40, gain_std=0.05)):
        fp = w.model_per_world == W.MODEL_FP
        w.params["Jp"][fp, 0] = 4e-9
        w.params["drag"][:] = DRAG
        _fd_check(w)


# ---- torque interface ------------------------------------------------------------------------

def test_torque_interface_hover_and_torque_response():
    """Collective thrust m g with zero torques hovers (allocation inverts the
    mixing); a small pure roll torque gives the initial body angular acceleration
    tau_x / J_x once the rotors reach their new commands."""
    b, P = fp_batch(1, control=O.CTRL_TORQUE)
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(17, 1, dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    u = torch.tensor([[W.MASS * W.GRAVITY], [0.0], [0.0], [0.0]], dtype=F64)
    y = run(b, x, u, 500)
    assert torch.allclose(y, x, atol=1e-9 * wh)
    # rotors held at the commanded speeds: torque about x from the mixing equals tau_x
    tau = 1e-5
    u2 = torch.tensor([[W.MASS * W.GRAVITY], [tau], [0.0], [0.0]], dtype=F64)
    rc = O.allocate(u2, b.P_fp)
    thrust, torque = O.rotor_wrench(rc, b.P_fp)
    assert abs(float(torque[0, 0]) - tau) < 1e-12 and abs(float(thrust[0]) - W.MASS * W.GRAVITY) < 1e-12
    assert abs(float(torque[1, 0])) < 1e-15 and abs(float(torque[2, 0])) < 1e-15


def test_gradient_fd_torque_interface():
    w = W.fp_torque(seed=25, n_worlds=3, steps=30)
    w.ref_offset = w.x0[0:3].copy()
    w.dloss = np.ones(3, np.float32)
    w.w_u = 1.0
    w.cmds = np.repeat(w.cmds[None], w.steps, axis=0)
    _fd_check(w, h=1e-6)


# ---- identified model without thrust dynamics (c_tau = 0) -----------------------------

def _direct(P):
    P["c_tau"][:] = 0.0


@pytest.mark.parametrize("integ", [O.RK4, O.EULER])
def test_direct_thrust_level_flight_closed_form(integ):
    """Level attitude, held thrust command f: the vertical acceleration is the
    constant c_f f / m - g, so z is the exact quadratic (RK4; Euler with its
    dt lag) and the thrust row holds f after every step, whatever it held before."""
    dt, n = 0.002, 400
    b, P = id_batch(2, integrator=integ, dt=dt, edit=_direct)
    x = torch.zeros(13, 2, dtype=F64)
    x[8] = torch.tensor([0.5, -1.0], dtype=F64)
    x[12] = torch.tensor([0.0, 1.0], dtype=F64)        # ignored by the direct variant
    f = torch.tensor([0.2, 0.4], dtype=F64)
    u = torch.stack([torch.zeros(2, dtype=F64)] * 3 + [f])
    y = run(b, x, u, n)
    t = n * dt
    a = W.ID_CF * f / W.MASS - W.GRAVITY
    z = x[8] * t + 0.5 * a * t * t
    if integ == O.EULER:
        z = z - 0.5 * a * t * dt
    assert torch.allclose(y[2], z, rtol=0, atol=1e-11)
    assert torch.equal(y[12], f)
    assert torch.allclose(y[8], x[8] + a * t, rtol=0, atol=1e-11)


def test_fast_thrust_lag_converges_to_direct_variant():
    """The 13-state model with a thrust time constant 1/c_tau -> 0 approaches the
    direct variant at first order in 1/c_tau."""
    dt, n = 1e-4, 2000
    rng = np.random.default_rng(3)
    x = torch.zeros(13, 3, dtype=F64)
    x[3:6] = torch.as_tensor(rng.uniform(-0.2, 0.2, (3, 3)))
    x[12] = W.MASS * W.GRAVITY
    u = torch.as_tensor(np.vstack([rng.uniform(-0.2, 0.2, (3, 3)), rng.uniform(0.2, 0.4, (1, 3))]))
    bd, _ = id_batch(3, dt=dt, edit=_direct)
    yd = run(bd, x, u, n)
    errs = []
    for ctau in (1e2, 1e3):
        b, _ = id_batch(3, dt=dt, edit=lambda P, c=ctau: P["c_tau"].__setitem__(slice(None), c))
        y = run(b, x, u, n)
        errs.append(float((y[0:12] - yd[0:12]).abs().max()))
    assert 8 < errs[0] / errs[1] < 12, errs


def test_gradient_fd_direct_thrust():
    w = W.id_rollout_grad(seed=26, n_worlds=3, steps=40)
    w.params["c_tau"][[0, 2]] = 0.0
    w.gain = w.gain * 5
    _fd_check(w)


# ---- position interface (geometric controller) ----------------------------------------

def _hover17(p):
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(17, 1, dtype=F64)
    x[0:3, 0] = torch.tensor(p, dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    return x, wh


def test_position_controller_hover_equilibrium():
    b, _ = fp_batch(1, control=O.CTRL_POSITION)
    x, _ = _hover17([0.3, -0.2, 1.0])
    u = torch.tensor([[0.3], [-0.2], [1.0], [0.0]], dtype=F64)
    y = run(b, x, u, 1000)
    assert float((y - x).abs().max()) < 1e-9


def test_position_controller_linearisation_is_stable():
    """Jacobian of the closed-loop discrete map at hover on the setpoint: with no
    integrator and every degree of freedom controlled, all modes lie strictly
    inside the unit circle."""
    b, _ = fp_batch(1, control=O.CTRL_POSITION)
    x, wh = _hover17([0.0, 0.0, 1.0])
    u = torch.tensor([[0.0], [0.0], [1.0], [0.0]], dtype=F64)
    scale = torch.ones(17, dtype=F64)
    scale[13:17] = wh
    Jm = torch.zeros(17, 17, dtype=F64)
    for j in range(17):
        h = 1e-6 * scale[j]
        xp, xm = x.clone(), x.clone()
        xp[j] += h
        xm[j] -= h
        Jm[:, j] = (b.step(xp, u) - b.step(xm, u))[:, 0] / (2 * h)
    keep = [i for i in range(17) if i != 6]
    mag = np.abs(np.linalg.eigvals(Jm[keep][:, keep].numpy()))
    assert mag.max() < 1 - 1e-3


def test_position_controller_reaches_setpoint_and_yaw():
    b, _ = fp_batch(1, control=O.CTRL_POSITION)
    x, _ = _hover17([0.3, 0.0, 1.0])
    u = torch.tensor([[1.3], [0.3], [1.5], [0.5]], dtype=F64)
    y = run(b, x, u, 5000)
    assert torch.allclose(y[0:3], u[0:3], atol=1e-4)
    qx, qy, qz, qw = (float(v) for v in y[3:7, 0])
    yaw = math.atan2(2 * (qw * qz + qx * qy), 1 - 2 * (qy * qy + qz * qz))
    assert abs(yaw - 0.5) < 1e-4
    assert float(y[7:13].abs().max()) < 1e-4


def test_position_controller_yaw_equivariance():
    """Rotating the start, the setpoint and the yaw setpoint about world z by a
    rotates the whole closed-loop trajectory by a."""
    b, _ = fp_batch(1, control=O.CTRL_POSITION)
    x, _ = _hover17([0.2, -0.4, 0.8])
    x[3:7, 0] = torch.tensor([0.05, -0.03, 0.1, 1.0], dtype=F64) / math.sqrt(1 + 0.05 ** 2 + 0.03 ** 2 + 0.01)
    x[7:13, 0] = torch.tensor([0.3, -0.1, 0.2, 0.5, -0.4, 0.3], dtype=F64)
    u = torch.tensor([[1.0], [0.5], [1.2], [0.3]], dtype=F64)
    a = 0.7
    Rz = torch.tensor([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]], dtype=F64)
    qz = torch.tensor([[0.0], [0.0], [math.sin(a / 2)], [math.cos(a / 2)]], dtype=F64)
    xr = x.clone()
    xr[0:3] = Rz @ x[0:3]
    xr[3:7] = O.quat_mul(qz, x[3:7])
    xr[7:10] = Rz @ x[7:10]
    ur = u.clone()
    ur[0:3] = Rz @ u[0:3]
    ur[3] = u[3] + a
    y, yr = run(b, x, u, 400), run(b, xr, ur, 400)
    assert torch.allclose(yr[0:3], Rz @ y[0:3], atol=1e-10)
    assert torch.allclose(yr[7:10], Rz @ y[7:10], atol=1e-10)
    assert torch.allclose(yr[3:7], O.quat_mul(qz, y[3:7]), atol=1e-10)
    assert torch.allclose(yr[10:17], y[10:17], atol=1e-8 * 15000)


def test_gradient_fd_position_interface():
    w = W.fp_position(seed=27, n_worlds=3, steps=30)
    w.ref_offset = w.cmds[0:3].copy()
    w.dloss = np.ones(3, np.float32)
    w.w_u = 1e-2
    w.cmds = np.repeat(w.cmds[None], w.steps, axis=0)
    _fd_check(w)


def test_binary32_storage_between_calls():
    """simulate_held(store_every=k) equals k-step fp64 runs chained through a
    binary32 copy of the state (the numpy cast is the definition of that rounding),
    and leaves every component representable in binary32."""
    w = W.small("fp_pid_closed_loop", seed=2)
    w = W.subset(w, list(range(6)))
    n, k = 12, 4
    got = O.simulate_held(w, steps=n, store_every=k).numpy()
    x = np.asarray(w.x0, np.float64)
    for _ in range(n // k):
        x = O.simulate_held(w, steps=k, x0=x).numpy().astype(np.float32).astype(np.float64)
    assert np.array_equal(got, x)
    assert np.array_equal(got.astype(np.float32).astype(np.float64), got)
    # storing only at the end is a rounding of the fp64 result
    full = O.simulate_held(w, steps=n).numpy()
    assert np.array_equal(O.simulate_held(w, steps=n, store_every=n).numpy(), full.astype(np.float32).astype(np.float64))


# ---- onboard controller at a lower rate than the physics ---------------------------

@pytest.mark.parametrize("n", [2, 5])
def test_multirate_controller_is_blocks_of_rotor_interface_steps(n):
    """With the controller every n physics steps, a run equals, block by block: the
    attitude PID evaluated once with period n dt, then n steps of the rotor
    interface under its commands, then the controller state it produced (built
    here from the rotor-interface path, not from the multirate step)."""
    w = W.small("fp_pid_closed_loop", seed=2)
    w = W.subset(w, list(range(8)))
    w.ctrl_every = n
    steps = 3 * n + 1
    got = O.simulate_held(w, steps=steps).numpy()
    b = O.Batch.from_workload(w)
    P = b.P_fp
    x = O.t64(w.x0)
    u = O.t64(w.cmds)
    t = 0
    with torch.no_grad():
        while t < steps:
            rot, cs = O.attitude_pid(x, u, P, n * b.dt)
            for _ in range(min(n, steps - t)):
                body = O.step_fp(x[0:17], rot, P, O.CTRL_ROTOR, b.integrator, b.dt, b.renorm)
                x = torch.cat([body, x[17:25]], 0)
                t += 1
            x = torch.cat([x[0:17], cs], 0)
    assert np.allclose(got, x.numpy(), rtol=0, atol=1e-14)


@pytest.mark.parametrize("control", [O.CTRL_TORQUE, O.CTRL_POSITION])
def test_multirate_torque_and_position_hold_commands(control):
    """Torque and position interfaces with the controller every 3 steps: the
    rotor commands of each evaluation drive three rotor-interface steps."""
    w = W.fp_torque(seed=31, n_worlds=5, steps=9) if control == O.CTRL_TORQUE else \
        W.fp_position(seed=32, n_worlds=5, steps=9)
    w.ctrl_every = 3
    got = O.simulate_held(w).numpy()
    b = O.Batch.from_workload(w)
    x, u = O.t64(w.x0), O.t64(w.cmds)
    with torch.no_grad():
        for t in range(w.steps):
            if t % 3 == 0:
                rot = O.allocate(u, b.P_fp) if control == O.CTRL_TORQUE else O.position_controller(x, u, b.P_fp)
            x = O.step_fp(x, rot, b.P_fp, O.CTRL_ROTOR, b.integrator, b.dt, b.renorm)
    assert np.allclose(got, x.numpy(), rtol=0, atol=1e-14)


def test_multirate_hover_fixed_point():
    """Hover with the attitude PID evaluated every 5 steps stays put."""
    b, P = fp_batch(2, control=O.CTRL_ATT_PID)
    b.ctrl_every = 5
    wh = math.sqrt(W.MASS * W.GRAVITY / (4 * W.K_THRUST))
    x = torch.zeros(25, 2, dtype=F64)
    x[6] = 1.0
    x[13:17] = wh
    u = torch.tensor([[0.0] * 2, [0.0] * 2, [0.0] * 2, [W.MASS * W.GRAVITY] * 2], dtype=F64)
    held = None
    y = x
    with torch.no_grad():
        for t in range(500):
            y, held = b.step_at(y, u, t, held)
    assert torch.allclose(y[0:13], x[0:13], atol=1e-11)
    assert torch.allclose(y[13:17], x[13:17], rtol=1e-12)
    assert torch.allclose(y[17:25], x[17:25], atol=1e-12)


def test_gradient_fd_multirate_controller():
    """Reverse-mode gradient through held controller outputs (PID every 3 steps)
    against central differences."""
    w = W.uneven_mixed_adjoint(seed=14, n_worlds=6, n_subset=4, steps=31, n_max=3)
    w.ctrl_every = 3
    _fd_check(w)


# ---- the BPTT tracking reward ----------------------------------------------------

def test_tilt_angle_matches_scipy():
    """Angle between the body and world z axes vs SciPy's rotations, for random
    quaternions (first principles) and ZYX Euler angles (identified)."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(5)
    n = 64
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    eul = rng.uniform(-1.2, 1.2, size=(n, 3))
    bf, _ = fp_batch(n, control=O.CTRL_ATT_PID)
    x = torch.zeros(25, n, dtype=F64)
    x[3:7] = torch.as_tensor(q.T)
    zf = Rotation.from_quat(q).apply([0.0, 0.0, 1.0])
    assert np.allclose(O.tilt_angle(bf, x).numpy(), np.arccos(np.clip(zf[:, 2], -1, 1)), atol=1e-7)
    wi = W.id_rollout_grad(seed=3, n_worlds=n, steps=1)
    bi = O.Batch.from_workload(wi)
    xi = torch.zeros(13, n, dtype=F64)
    xi[3:6] = torch.as_tensor(eul.T)
    zi = Rotation.from_euler("ZYX", eul[:, ::-1]).apply([0.0, 0.0, 1.0])
    assert np.allclose(O.tilt_angle(bi, xi).numpy(), np.arccos(np.clip(zi[:, 2], -1, 1)), atol=1e-7)


def _hover_on_reference(w):
    """Hover at the reference point with the hover action: amplitude-0 reference
    centred on each drone, zero velocity, no feedback."""
    b = O.Batch.from_workload(w)
    a = O.hover_action(b).numpy()
    w.ref_amp = 0.0
    w.ref_offset = w.x0[0:3].copy()
    w.gain = None
    w.cmds = np.repeat(a[None], w.steps, 0).astype(np.float32)
    return w


@pytest.mark.parametrize("model", ["id", "fp_pid"])
def test_reward_is_one_per_step_in_hover_on_the_reference(model):
    if model == "id":
        w = W.id_rollout_grad(seed=7, n_worlds=5, steps=20)
        w.x0[6:9] = 0.0
        w.x0[3:6] = 0.0
        w.x0[12] = W.MASS * W.GRAVITY / W.ID_CF
    else:
        w = W.fp_pid_closed_loop(seed=7, n_worlds=5, steps=20)
        w.x0[3:7] = np.array([0, 0, 0, 1.0])[:, None]
        w.x0[7:13] = 0.0
        w.x0[17:25] = 0.0
    w = _hover_on_reference(w)
    w.reward = W.BPTT_REWARD
    out = O.rollout_workload(w)
    assert np.allclose(out["loss"].numpy(), -w.steps, atol=1e-9)


def test_smoothness_term_telescopes_for_a_held_action():
    """With the same action at every step the smoothness penalty is paid once,
    against the hover action before the first step."""
    w = W.id_rollout_grad(seed=8, n_worlds=4, steps=15)
    w.gain = None
    a = O.hover_action(O.Batch.from_workload(w)).numpy() + np.array([0.05, -0.03, 0.02, 0.01])[:, None]
    w.cmds = np.repeat(a[None], w.steps, 0).astype(np.float32)
    r0 = dict(W.BPTT_REWARD, w_dact=[0.0] * 4)
    r1 = dict(W.BPTT_REWARD, w_dact=[1.0, 2.0, 3.0, 4.0])
    w.reward = r0
    l0 = O.rollout_workload(w)["loss"].numpy()
    w.reward = r1
    l1 = O.rollout_workload(w)["loss"].numpy()
    da = w.cmds[0].astype(np.float64) - O.hover_action(O.Batch.from_workload(w)).numpy()
    assert np.allclose(l1 - l0, (np.array(r1["w_dact"])[:, None] * da ** 2).sum(0), rtol=1e-12, atol=1e-12)


def _tilted(w, seed):
    """Start every drone tilted (0.05-0.15 rad) so the tilt term stays away from
    its kink at the upright orientation, where differences are not derivatives."""
    rng = np.random.default_rng(seed)
    x0 = w.x0.astype(np.float64)
    D = x0.shape[1]
    ang = rng.uniform(0.05, 0.15, size=D) * rng.choice([-1.0, 1.0], size=(2, D))
    if x0.shape[0] >= 17:
        world = np.repeat(np.arange(w.n_worlds), w.drones_per_world)
        fp = w.model_per_world[world] == W.MODEL_FP
        q = np.stack([np.sin(ang[0] / 2), np.sin(ang[1] / 2), np.zeros(D), np.ones(D)])
        q /= np.linalg.norm(q, axis=0, keepdims=True)
        x0[3:7, fp] = q[:, fp]
        x0[3:5, ~fp] = ang[:, ~fp]
    else:
        x0[3:5] = ang
    w.x0 = x0.astype(np.float32)
    return w


def test_gradient_fd_reward_identified():
    w = W.small("id_rollout_grad", seed=16)
    w.steps = 40
    w.cmds = w.cmds[:40]
    w.reward = W.BPTT_REWARD
    _fd_check(_tilted(w, 16), h=1e-5)


def test_gradient_fd_reward_first_principles_pid():
    w = W.uneven_mixed_adjoint(seed=17, n_worlds=6, n_subset=4, steps=30, n_max=3)
    w.reward = W.BPTT_REWARD
    _fd_check(_tilted(w, 17), h=3e-6)


# ---- the figure-eight reference of the tracking objective (reading r19) -----------------

def _eight_batch():
    """Two first-principles and two identified single-drone worlds with distinct
    masses and thrust scalings, so per-drone reference rows are told apart."""
    n = 4
    P = W.empty_params(n)
    masses = np.array([0.027, 0.031, 0.024, 0.035])
    W.fill_fp_airframe(P, np.arange(2), masses[:2], np.tile(W.INERTIA, (2, 1)))
    W.fill_id_model(P, np.arange(2, 4), np.tile(W.ID_GAIN, (2, 1)), np.tile(W.ID_TAU, (2, 1)))
    P["mass"][2:4, 0] = masses[2:]
    P["c_f"][2:4, 0] = [0.9, 1.2]
    b = O.Batch(np.ones(n, np.int64), np.array([0, 0, 1, 1]), P, O.CTRL_ATT_PID, O.RK4, 0.002)
    b.params_in = P
    return b, masses


def test_figure_eight_passes_its_quarter_points():
    """A sin(2 pi t/P), (A/2) sin(4 pi t/P): through the origin at t = 0 and P/2,
    at (A/sqrt2, +-A/2) at t = P/8 and 3P/8, at (A, 0) at t = P/4; there the
    curve moves along -y at speed 2 pi A/P, and through the origin at t = 0 it
    moves along the diagonal (1, 1) at speed 2 sqrt2 pi A/P."""
    b, _ = _eight_batch()
    A, Pd = 1.3, 4.0
    s = 1.0 / math.sqrt(2.0)
    pts = {0.0: (0.0, 0.0), Pd / 8: (A * s, A / 2), Pd / 4: (A, 0.0), 3 * Pd / 8: (A * s, -A / 2),
           Pd / 2: (0.0, 0.0)}
    for t, (x, y) in pts.items():
        p, _ = b.figure_eight(t, A, Pd, None)
        assert torch.allclose(p[:, 0], torch.tensor([x, y, 0.0], dtype=F64), atol=1e-14), t
    w0 = 2 * math.pi / Pd
    _, v = b.figure_eight(Pd / 4, A, Pd, None)
    assert torch.allclose(v[:, 0], torch.tensor([0.0, -A * w0, 0.0], dtype=F64), atol=1e-13)
    _, v = b.figure_eight(0.0, A, Pd, None)
    assert torch.allclose(v[:, 0], torch.tensor([A * w0, A * w0, 0.0], dtype=F64), atol=1e-13)
    _, v = b.figure_eight(Pd / 2, A, Pd, None)
    assert torch.allclose(v[:, 0], torch.tensor([-A * w0, A * w0, 0.0], dtype=F64), atol=1e-13)


def test_figure_eight_is_a_periodic_gerono_lemniscate():
    """Every point satisfies the lemniscate of Gerono's implicit equation
    y^2 = x^2 (1 - x^2 / A^2) with z = 0, and p(t + P) = p(t)."""
    b, _ = _eight_batch()
    A, Pd = 0.8, 3.0
    for t in np.random.default_rng(3).uniform(0.0, 10.0, 40):
        p, _ = b.figure_eight(float(t), A, Pd, None)
        x, y, z = (float(c) for c in p[:, 0])
        assert abs(y * y - x * x * (1.0 - x * x / (A * A))) <= 1e-14
        assert z == 0.0
        p2, _ = b.figure_eight(float(t) + Pd, A, Pd, None)
        assert torch.allclose(p, p2, atol=1e-13)


def test_figure_eight_velocity_is_the_derivative_of_the_position():
    """v_ref equals a central difference of p_ref (h = 1e-5: truncation ~1e-10)."""
    b, _ = _eight_batch()
    A, Pd, h = 1.0, 4.0, 1e-5
    for t in np.random.default_rng(4).uniform(0.0, 8.0, 25):
        t = float(t)
        _, v = b.figure_eight(t, A, Pd, None)
        pp, _ = b.figure_eight(t + h, A, Pd, None)
        pm, _ = b.figure_eight(t - h, A, Pd, None)
        assert torch.allclose((pp - pm) / (2 * h), v, atol=1e-8)


def test_figure_eight_offset_translates_position_only():
    b, _ = _eight_batch()
    off = torch.as_tensor(np.random.default_rng(5).normal(size=(3, 4)))
    p0, v0 = b.figure_eight(0.7, 1.0, 4.0, None)
    p1, v1 = b.figure_eight(0.7, 1.0, 4.0, off)
    assert torch.allclose(p1 - p0, off, atol=1e-15)
    assert torch.equal(v1, v0)


def test_reference_state_rows_per_model():
    """First principles: [p, (0, 0, 0, 1), v, 0]; identified: [p, 0, v, 0, m g / c_f]
    with each drone's own mass and thrust scaling (reading r18). Hover check: an
    identified drone at its reference thrust state with the level attitude and
    zero velocity keeps its altitude (the thrust row balances gravity)."""
    b, masses = _eight_batch()
    p, v = b.figure_eight(1.1, 1.0, 4.0, None)
    xr = b.reference_state(p, v)
    for d in range(2):
        assert torch.equal(xr[0:3, d], p[:, d])
        assert torch.equal(xr[3:7, d], torch.tensor([0.0, 0.0, 0.0, 1.0], dtype=F64))
        assert torch.equal(xr[7:10, d], v[:, d])
        assert torch.equal(xr[10:13, d], torch.zeros(3, dtype=F64))
    for d, cf in ((2, 0.9), (3, 1.2)):
        assert torch.equal(xr[0:3, d], p[:, d])
        assert torch.equal(xr[3:6, d], torch.zeros(3, dtype=F64))
        assert torch.equal(xr[6:9, d], v[:, d])
        assert torch.equal(xr[9:12, d], torch.zeros(3, dtype=F64))
        assert abs(float(xr[12, d]) - masses[d] * W.GRAVITY / cf) <= 1e-15
    # the identified drones at [p, 0, 0, 0, f_ref] with command [0, 0, 0, f_ref] hover
    x = torch.zeros(13, 4, dtype=F64)
    x[12] = xr[12]
    x = x[:, 2:4]
    bi = O.Batch(np.ones(2, np.int64), np.ones(2), {k: v_[2:4] for k, v_ in b.params_in.items()},
                 O.CTRL_ATT_PID, O.RK4, 0.002)
    u = torch.zeros(4, 2, dtype=F64)
    u[3] = x[12]
    y = run(bi, x.clone(), u, 50)
    assert torch.allclose(y, x, atol=1e-12)


# ---- the small-MLP policy of the BPTT setup (reading r30) -------------------------------

def test_mlp_policy_with_small_weights_is_the_linear_feedback():
    """With W1 = eps A, W2 = B, W3 = C and zero biases the MLP output is
    eps C B A e + O(eps^3): the rollout converges to the one with the linear
    gain eps C B A at second order in eps (relative)."""
    w = W.id_rollout_grad_mlp(seed=40, n_worlds=6, steps=60, hidden=8)
    H = 8
    rng = np.random.default_rng(40)
    A = rng.normal(size=(H, 13))
    Bm = rng.normal(size=(H, H)) / math.sqrt(H)
    C = rng.normal(size=(4, H)) * 0.3
    b = O.Batch.from_workload(w)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u)
    errs = []
    for eps in (0.02, 0.01, 0.005):
        theta = np.concatenate([(eps * A).ravel(), np.zeros(H), Bm.ravel(), np.zeros(H), C.ravel(), np.zeros(4)])
        G = (eps * C @ Bm @ A)[None]
        with torch.no_grad():
            m = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, gain=torch.as_tensor(theta)[None],
                          policy_hidden=H, **kw)
            l = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, gain=torch.as_tensor(G), **kw)
        # compare the feedback's effect: trajectories differ from the open loop by O(eps)
        errs.append(float((m["x"] - l["x"]).abs().max()))
    assert errs[0] / errs[1] > 6.0 and errs[1] / errs[2] > 6.0, errs   # third order in eps


def test_mlp_policy_output_layer_gradient_identity():
    """u_t = ubar_t + W3 h2_t + b3 gives dL/dW3 = sum_t (dL/du_t) h2_t^T and
    dL/db3 = sum_t dL/du_t exactly."""
    w = W.id_rollout_grad_mlp(seed=41, n_worlds=3, steps=25, hidden=6, out_scale=0.05)
    H = 6
    b = O.Batch.from_workload(w)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period, w_u=w.w_u, policy_hidden=H)
    theta = O.t64(w.gain)
    g = O.rollout_grad(b, w.x0, w.cmds, w.steps, gain=theta, dloss=w.dloss, **kw)
    out = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, gain=theta, keep_traj=True, **kw)
    traj = out["traj"].detach()
    P = O.mlp_param_count(H)
    th = theta[0]
    W1 = th[:13 * H].reshape(H, 13); b1 = th[13 * H:14 * H]
    W2 = th[14 * H:14 * H + H * H].reshape(H, H); b2 = th[14 * H + H * H:15 * H + H * H]
    accW, accb = torch.zeros(4, H, dtype=F64), torch.zeros(4, dtype=F64)
    for n in range(w.steps):
        p, v = b.figure_eight(n * b.dt, w.ref_amp, w.ref_period, None)
        e = traj[n, 0:13] - b.reference_state(p, v)
        h2 = torch.tanh(W2 @ torch.tanh(W1 @ e + b1[:, None]) + b2[:, None])
        accW += g["g_cmds"][n] @ h2.T
        accb += g["g_cmds"][n].sum(1)
    gth = g["g_gain"][0]
    assert torch.allclose(accW, gth[P - 4 - 4 * H:P - 4].reshape(4, H), rtol=1e-10, atol=1e-14)
    assert torch.allclose(accb, gth[P - 4:], rtol=1e-10, atol=1e-14)


def test_gradient_fd_mlp_policy():
    w = W.id_rollout_grad_mlp(seed=42, n_worlds=3, steps=20, hidden=5, out_scale=0.05)
    _fd_check(w)


def test_reference_time_offset_equals_the_shifted_table():
    """A rollout that follows the figure-eight from step k equals the same rollout
    given the reference rows of steps k .. k + T as an explicit table."""
    w = W.id_rollout_grad(seed=43, n_worlds=4, steps=30)
    k = 777
    b = O.Batch.from_workload(w)
    rows = []
    for n in range(w.steps + 1):
        p, v = b.figure_eight((k + n) * b.dt, w.ref_amp, w.ref_period, None)
        rows.append(b.reference_state(p, v)[:, 0])
    table = torch.stack(rows)
    kw = dict(gain=O.t64(w.gain), w_u=w.w_u)
    with torch.no_grad():
        a = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, ref_amp=w.ref_amp, ref_period=w.ref_period,
                      ref_step0=k, **kw)
        c = O.rollout(b, O.t64(w.x0), O.t64(w.cmds), w.steps, ref_table=table, **kw)
    assert torch.allclose(a["loss"], c["loss"], rtol=1e-12, atol=0)
    assert torch.allclose(a["x"], c["x"], rtol=1e-12, atol=1e-15)


def test_reference_time_shift_equals_per_drone_start_steps():
    """A per-drone time shift of k_d steps equals following the figure-eight from
    step k_d (dt a power of two, so k dt is exact in both forms), drone by drone,
    with the linear feedback, per-drone offsets and both objectives."""
    w = W.id_rollout_grad(seed=44, n_worlds=5, steps=30, dt=2.0 ** -9)
    ks = np.array([0, 3, 250, 1024, 4095])
    w.ref_offset = W._f32(np.random.Generator(np.random.Philox(44)).normal(0.0, 0.3, size=(3, 5)))
    w.ref_time_shift = (ks * w.dt).astype(np.float32)
    assert np.array_equal(w.ref_time_shift.astype(np.float64), ks * w.dt)
    for reward in (None, W.BPTT_REWARD):
        w.reward = reward
        both = O.rollout_workload(w)
        for d, k in enumerate(ks):
            one = W.subset(w, [d])
            one.ref_time_shift = None
            one.ref_step0 = int(k)
            r = O.rollout_workload(one)
            assert torch.allclose(both["loss"][d:d + 1], r["loss"], rtol=1e-13, atol=1e-13), (reward, d)
            assert torch.allclose(both["x"][:, d:d + 1], r["x"], rtol=1e-13, atol=1e-13), (reward, d)


def test_reference_time_shift_of_one_period_is_no_shift():
    w = W.id_rollout_grad(seed=45, n_worlds=3, steps=40)
    base = O.rollout_workload(w)
    w.ref_time_shift = np.full(3, w.ref_period, np.float32)
    r = O.rollout_workload(w)
    assert torch.allclose(base["loss"], r["loss"], rtol=1e-10, atol=0)
    assert torch.allclose(base["x"], r["x"], rtol=1e-10, atol=1e-12)


def test_bptt_tracking_starts_on_the_reference():
    """The BPTT setup's starts: position and velocity equal the figure-eight at each
    drone's time shift (closed form), hover thrust, level attitude."""
    w = W.bptt_tracking(n_envs=8, period=10.0)
    s = w.ref_time_shift.astype(np.float64)
    assert np.allclose(s, np.arange(8) * 10.0 / 8)
    w0 = 2 * math.pi / 10.0
    assert np.allclose(w.x0[0], np.sin(w0 * s), atol=1e-6)
    assert np.allclose(w.x0[1], 0.5 * np.sin(2 * w0 * s), atol=1e-6)
    assert np.allclose(w.x0[6], w0 * np.cos(w0 * s), atol=1e-6)
    assert np.allclose(w.x0[7], w0 * np.cos(2 * w0 * s), atol=1e-6)
    assert np.all(w.x0[[2, 3, 4, 5, 8, 9, 10, 11]] == 0)
    assert np.allclose(w.x0[12], W.MASS * W.GRAVITY / W.ID_CF)
    # hover thrust and a zero policy: no acceleration, so after one step the error
    # is the reference's own curvature, |a_ref| dt^2 / 2 <= sqrt(5) A w^2 dt^2 / 2
    r = O.rollout_workload(dataclasses.replace(w, steps=1, reward=None, w_u=0.0))
    bound = 0.5 * math.sqrt(5.0) * w0 ** 2 * w.dt ** 2
    assert float(r["loss"].max()) <= (1.01 * bound) ** 2
    assert float(r["loss"].max()) > (0.5 * bound) ** 2


def _squash_case(scale, gain_mult=1.0, steps=20, hidden=0):
    w = W.id_rollout_grad(seed=46, n_worlds=6, steps=steps)
    if hidden:
        w = W.id_rollout_grad_mlp(seed=46, n_worlds=6, steps=steps, hidden=hidden, out_scale=0.3)
    w.gain = W._f32(w.gain * gain_mult)
    w.policy_scale = None if scale is None else W._f32(scale)
    return w


def test_squashed_policy_small_output_limit_is_the_scaled_linear_policy():
    """s tanh(o) = s o - s o^3 / 3 + ...: with the gain shrunk by eps the squashed
    rollout and the unsquashed rollout with gain diag(s) G differ at third order in
    eps (halving eps divides the gap by 8)."""
    s = np.array([0.5, 0.4, 0.3, 0.2])
    gaps = []
    for eps in (0.1, 0.05, 0.025):
        w1 = _squash_case(s, gain_mult=eps * 20.0)
        w2 = _squash_case(None, gain_mult=eps * 20.0)
        w2.gain = w1.gain.astype(np.float64) * s[None, :, None]   # exact, not rounded to binary32
        a, b = O.rollout_workload(w1), O.rollout_workload(w2)
        base = O.rollout_workload(_squash_case(None, gain_mult=0.0))
        gaps.append(float((a["loss"] - b["loss"]).abs().max()))
        assert float((a["loss"] - base["loss"]).abs().max()) > 100 * gaps[-1]
    assert 7.0 < gaps[0] / gaps[1] < 9.0 and 7.5 < gaps[1] / gaps[2] < 8.5, gaps


def test_squashed_policy_saturates_at_the_range():
    """A huge gain saturates tanh: the first applied command is ubar + s sign(G e),
    i.e. one step equals the plain step under that command."""
    s = np.array([0.3, 0.2, 0.1, 0.05])
    w = _squash_case(s, gain_mult=1e7, steps=1)
    b = O.Batch.from_workload(w)
    x0 = O.t64(w.x0)
    p, v = b.figure_eight(0.0, w.ref_amp, w.ref_period, None)
    e = x0[0:13] - b.reference_state(p, v)
    o = (O.t64(w.gain)[0][None] * e.T[:, None, :]).sum(2).T
    assert float(o.abs().min()) > 40.0        # tanh(40) is 1 in binary64
    u = O.t64(w.cmds[0]) + O.t64(w.policy_scale)[:, None] * torch.sign(o)
    r = O.rollout_workload(w)
    x1, _ = b.step_at(x0, u, 0, None)
    assert torch.allclose(r["x"], x1, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("hidden", [0, 6])
def test_squashed_policy_gradients_match_central_differences(hidden):
    w = _squash_case(np.array([0.5, 0.5, 0.5, 0.2]), steps=15, hidden=hidden, gain_mult=1.0 if hidden else 30.0)
    w.reward = W.BPTT_REWARD
    w = _tilted(w, 47 + hidden)
    g = O.rollout_workload(w, with_grad=True)
    rng = np.random.Generator(np.random.Philox(47))
    for key, arr in (("g_gain", "gain"), ("g_cmds", "cmds"), ("g_x0", "x0")):
        base = getattr(w, arr).astype(np.float64)
        dirn = rng.normal(size=base.shape)
        h = 1e-6
        vals = []
        for sgn in (1, -1):
            wp = dataclasses.replace(w, **{arr: base + sgn * h * dirn})
            vals.append(float((O.rollout_workload(wp)["loss"] * O.t64(w.dloss)).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float((g[key] * O.t64(dirn)).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (key, fd, an)
