"""FP64 CPU oracle of the batched drone step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and its
Python binding) never calls it and shares no code with it.

What it computes (Crazyflow, arXiv 2606.01478, Methods):
  * first-principles model -- rigid body of Eq. (1) (position, scalar-last
    quaternion, velocity, body rate) driven by four rotors whose thrust and drag
    torque are second-order polynomials in rotor speed, combined through the
    x-configuration mixing matrix, and rotor speeds that follow the adapted,
    direction-dependent rotor dynamics (Eq. rotor_adapted) -- section
    "First Principles Modeling";
  * identified attitude-command model -- point mass pushed by a first-order
    collective-thrust state along R(Psi) e_z and a second-order linear attitude
    response (Eqs. 3_simplified_*) -- section "Abstracted Physics Modeling";
  * a cascaded attitude -> body-rate PID in front of the first-principles model
    for the attitude interface (the paper names the interface and the
    re-implemented onboard stack, not its gains; structure and gains here are
    this project's own design, see ``attitude_pid``);
  * explicit Euler / classical RK4 integration with the command held over the
    step (the paper integrates the equations of motion directly, without a
    solver loop -- section "Architecture"), quaternion renormalisation after
    every step;
  * a tracking rollout with optional linear state feedback and the loss
    sum_t |p_t - p_ref(t)|^2 + w_u sum_t |u_t|^2, and its exact reverse-mode
    gradient (PyTorch autograd on this same FP64 discrete map).

Everything is float64 on the CPU, vectorised over drones (tensors ``[k, D]``)
with a plain Python loop over time steps. Readings of the paper where it is
silent or garbled are listed next to the function that takes them.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

F64 = torch.float64

# enum values of the public interface
MODEL_FP, MODEL_ID = 0, 1
CTRL_ROTOR, CTRL_ATT_PID, CTRL_TORQUE, CTRL_POSITION = 0, 1, 2, 3
EULER, RK4 = 0, 1


# ---- helpers ------------------------------------------------------------------

def t64(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(F64)
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def per_drone_params(params: Dict[str, np.ndarray], drones_per_world) -> Dict[str, torch.Tensor]:
    """World parameter records ``[M, k]`` -> per-drone rows ``[k, D]`` (float64)."""
    world = np.repeat(np.arange(len(drones_per_world)), np.asarray(drones_per_world))
    return {k: torch.as_tensor(np.asarray(v, np.float64)[world].T.copy()) for k, v in params.items()}


def quat_mul(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Hamilton product of scalar-last quaternions ``[4, D]`` (reading: Hamilton
    convention, as in SciPy's Rotation, which the authors contributed to)."""
    av, aw = a[0:3], a[3]
    bv, bw = b[0:3], b[3]
    vec = aw * bv + bw * av + torch.linalg.cross(av, bv, dim=0)
    return torch.cat([vec, (aw * bw - (av * bv).sum(0))[None]], 0)


def body_z_in_world(q: torch.Tensor) -> torch.Tensor:
    """Third column of the body->world rotation matrix of a unit quaternion
    (x, y, z, w). Reading: inside RK4 stages the stage quaternion is used as is
    (no normalisation), with this unit-quaternion formula."""
    qx, qy, qz, qw = q[0], q[1], q[2], q[3]
    return torch.stack([2 * (qx * qz + qw * qy),
                        2 * (qy * qz - qw * qx),
                        1 - 2 * (qx * qx + qy * qy)])


def rotation_matrix(q: torch.Tensor) -> torch.Tensor:
    """Body->world rotation matrix [3, 3, D] of a unit quaternion (x, y, z, w),
    applied (like body_z_in_world) to the stage quaternion as is."""
    qx, qy, qz, qw = q[0], q[1], q[2], q[3]
    return torch.stack([
        torch.stack([1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)]),
        torch.stack([2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)]),
        torch.stack([2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)]),
    ])


def euler_zyx_matrix(psi: torch.Tensor) -> torch.Tensor:
    """R = Rz(yaw) Ry(pitch) Rx(roll) as [3, 3, D]."""
    phi, th, ps = psi[0], psi[1], psi[2]
    cf, sf, ct, st, cp, sp = torch.cos(phi), torch.sin(phi), torch.cos(th), torch.sin(th), torch.cos(ps), torch.sin(ps)
    return torch.stack([
        torch.stack([cp * ct, cp * st * sf - sp * cf, cp * st * cf + sp * sf]),
        torch.stack([sp * ct, sp * st * sf + cp * cf, sp * st * cf - cp * sf]),
        torch.stack([-st, ct * sf, ct * cf]),
    ])


def drag_acceleration(R: torch.Tensor, v: torch.Tensor, P) -> torch.Tensor:
    """R C_a R^T v / m: linear drag C_a v_body in the body frame, rotated to the world."""
    vb = (R * v[:, None, :]).sum(0)               # R^T v
    fb = P["drag"] * vb
    return (R * fb[None, :, :]).sum(1) / P["mass"][0]


def euler_zyx_body_z(psi: torch.Tensor) -> torch.Tensor:
    """R(Psi) e_z for R = Rz(yaw) Ry(pitch) Rx(roll) (reading: ZYX Euler angles)."""
    phi, th, ps = psi[0], psi[1], psi[2]
    return torch.stack([torch.cos(ps) * torch.sin(th) * torch.cos(phi) + torch.sin(ps) * torch.sin(phi),
                        torch.sin(ps) * torch.sin(th) * torch.cos(phi) - torch.cos(ps) * torch.sin(phi),
                        torch.cos(th) * torch.cos(phi)])


# ---- first-principles model -----------------------------------------------------

def rotor_rates(rot: torch.Tensor, rot_cmd: torch.Tensor, P) -> torch.Tensor:
    """Eq. rotor_adapted: the 'hat' coefficients apply when the command is at least
    the current speed (ties take that branch), the 'check' ones otherwise."""
    up = rot_cmd >= rot
    cv = torch.where(up, P["motor_up"][0:1], P["motor_down"][0:1])
    cd = torch.where(up, P["motor_up"][1:2], P["motor_down"][1:2])
    return cv * (rot_cmd - rot) + cd * (rot_cmd * rot_cmd - rot * rot)


def rotor_wrench(rot: torch.Tensor, P):
    """Per-rotor thrust and drag torque (second-order polynomials in the rotor
    speed), combined into collective thrust and body torques through the mixing
    matrix (rows tau_x, tau_y from the motor positions of the x airframe, tau_z
    from the spin directions)."""
    k0, k1, k2 = P["thrust_poly"][0:1], P["thrust_poly"][1:2], P["thrust_poly"][2:3]
    t0, t1, t2 = P["torque_poly"][0:1], P["torque_poly"][1:2], P["torque_poly"][2:3]
    f = k0 + k1 * rot + k2 * rot * rot
    tq = t0 + t1 * rot + t2 * rot * rot
    thrust = f.sum(0)
    torque = torch.stack([(P["mix_tx"] * f).sum(0),
                          (P["mix_ty"] * f).sum(0),
                          (P["mix_yaw"] * tq).sum(0)])
    return thrust, torque


def fp_rates(x: torch.Tensor, rot_cmd: torch.Tensor, P) -> torch.Tensor:
    """Time derivative of the 17-component first-principles state
    [p, q(x,y,z,w), v, w_body, Omega(4)] under rotor-speed command ``rot_cmd``.

    Eq. (1): p' = v; q' = 1/2 q (x) [w; 0]; m v' = f_sum; J w' = t_sum - w x J w,
    with f_sum = R(q) [0, 0, sum f_i] + R(q) C_a R(q)^T v - m g e_z (gravity along
    -z, g from the record; linear body-frame drag f_a = C_a v_body, C_a diagonal)
    and t_sum = mixed rotor torques + gyroscopic/reaction torques of the rotors.

    Reading of the garbled gyroscopic rows: rotor i spins with direction
    sigma_i = -sign(mix_yaw_i) (+,-,+,- for the x airframe), so the rotors carry
    angular momentum h = J_p Omega_s e_z, Omega_s = sum sigma_i Omega_i, and
    Euler's equation with internal rotors adds -w x h - h' =
    J_p [-w_y Omega_s, w_x Omega_s, -sum sigma_i Omega_i'] to the torques; the
    third row is the reaction torque exactly as printed.
    """
    q, v, w, rot = x[3:7], x[7:10], x[10:13], x[13:17]
    rot_dot = rotor_rates(rot, rot_cmd, P)
    thrust, torque = rotor_wrench(rot, P)
    m, g = P["mass"][0], P["gravity"][0]
    acc = (thrust / m) * body_z_in_world(q)
    acc = acc - torch.stack([torch.zeros_like(g), torch.zeros_like(g), g])
    acc = acc + drag_acceleration(rotation_matrix(q), v, P)
    sigma = -torch.sign(P["mix_yaw"])
    jp = P["Jp"][0]
    om_s = (sigma * rot).sum(0)
    torque = torque + jp * torch.stack([-w[1] * om_s, w[0] * om_s, -(sigma * rot_dot).sum(0)])
    q_dot = 0.5 * quat_mul(q, torch.cat([w, torch.zeros_like(w[0:1])], 0))
    J = P["J"]
    w_dot = (torque - torch.linalg.cross(w, J * w, dim=0)) / J
    return torch.cat([v, q_dot, acc, w_dot, rot_dot], 0)


def roll_pitch_from_quat(q: torch.Tensor):
    """Roll and pitch of the ZYX Euler decomposition of a unit quaternion."""
    qx, qy, qz, qw = q[0], q[1], q[2], q[3]
    roll = torch.atan2(2 * (qw * qx + qy * qz), 1 - 2 * (qx * qx + qy * qy))
    pitch = torch.asin(torch.clamp(2 * (qw * qy - qz * qx), -1.0, 1.0))
    return roll, pitch


def rotor_speed_for_thrust(f: torch.Tensor, P) -> torch.Tensor:
    """Positive root of k0 + k1 W + k2 W^2 = f (k2 > 0). Where the discriminant
    is not positive (zero thrust with k0 = k1 = 0) the root is -k1/(2 k2) and its
    gradient is taken as zero (the true slope is infinite there)."""
    k0, k1, k2 = P["thrust_poly"][0:1], P["thrust_poly"][1:2], P["thrust_poly"][2:3]
    disc = k1 * k1 - 4 * k2 * (k0 - f)
    pos = disc > 0
    root = torch.sqrt(torch.where(pos, disc, torch.ones_like(disc)))
    return torch.where(pos, (root - k1) / (2 * k2), -k1 / (2 * k2) + 0 * disc)


def attitude_pid(x: torch.Tensor, u: torch.Tensor, P, dt: float):
    """Attitude interface of the first-principles model: command
    u = [roll, pitch, yaw rate, collective thrust].

    The paper re-implements the Crazyflie onboard stack but prints no structure
    or gains; this project's controller (evaluated once per physics step, at the
    start of the step) is:
      e_a = [roll_c - roll, pitch_c - pitch]        I_a += e_a dt
      rate_sp = [kp_a e_a + ki_a I_a, yawrate_c]
      e_r = rate_sp - w                             I_r += e_r dt
      alpha = kp_r e_r + ki_r I_r - kd_r (w - w_prev)/dt     w_prev <- w
      [f_1..f_4] = clamp(alloc [T_c, J_ctrl alpha], 0, f_max)
      Omega_cmd_i = rotor speed giving f_i on the thrust curve.
    Controller state (8): I_a(2), I_r(3), w_prev(3) in rows 17..24.
    """
    roll, pitch = roll_pitch_from_quat(x[3:7])
    w = x[10:13]
    i_ang, i_rate, w_prev = x[17:19], x[19:22], x[22:25]
    e_ang = torch.stack([u[0] - roll, u[1] - pitch])
    i_ang = i_ang + e_ang * dt
    rate_sp = torch.cat([P["ang_kp"] * e_ang + P["ang_ki"] * i_ang, u[2:3]], 0)
    e_rate = rate_sp - w
    i_rate = i_rate + e_rate * dt
    alpha = P["rate_kp"] * e_rate + P["rate_ki"] * i_rate - P["rate_kd"] * (w - w_prev) / dt
    wrench = torch.cat([u[3:4], P["J_ctrl"] * alpha], 0)
    return allocate(wrench, P), torch.cat([i_ang, i_rate, w], 0)


def position_controller(x: torch.Tensor, u: torch.Tensor, P) -> torch.Tensor:
    """Position interface of the first-principles model: command u = [x, y, z,
    yaw] setpoints, a geometric controller on SO(3) of the kind the paper
    provides for its trajectory tracking (after Mellinger and Kumar; the paper
    names it and says it needs only the mass; the structure below and its gains
    are this project's design):
      a = -kp (p - p_sp) - kv v + g e_z,   F = m a
      T = F . (R e_z)                      (collective thrust along the body z)
      z_d = F / |F|,  y_d = z_d x [cos yaw, sin yaw, 0] normalised,  x_d = y_d x z_d
      e_R = vee(R_d^T R - R^T R_d) / 2,    e_w = w (rate setpoint zero)
      tau = J_ctrl (-kR e_R - kw e_w)
    then the attitude controller's allocation. No controller state."""
    p, q, v, w = x[0:3], x[3:7], x[7:10], x[10:13]
    m, g = P["mass"][0], P["gravity"][0]
    zero = torch.zeros_like(g)
    a = -P["pos_kp"] * (p - u[0:3]) - P["pos_kv"] * v + torch.stack([zero, zero, g])
    F = m * a
    R = rotation_matrix(q)
    T = (F * R[:, 2]).sum(0)
    z_d = F / torch.sqrt((F * F).sum(0))
    x_c = torch.stack([torch.cos(u[3]), torch.sin(u[3]), torch.zeros_like(u[3])])
    y_d = torch.linalg.cross(z_d, x_c, dim=0)
    y_d = y_d / torch.sqrt((y_d * y_d).sum(0))
    x_d = torch.linalg.cross(y_d, z_d, dim=0)
    Rd = torch.stack([x_d, y_d, z_d], 1)                          # columns
    E = torch.einsum("jid,jkd->ikd", Rd, R) - torch.einsum("jid,jkd->ikd", R, Rd)
    e_R = 0.5 * torch.stack([E[2, 1], E[0, 2], E[1, 0]])
    tau = P["J_ctrl"] * (-P["att_kr"] * e_R - P["att_kw"] * w)
    return allocate(torch.cat([T[None], tau], 0), P)


def allocate(wrench: torch.Tensor, P) -> torch.Tensor:
    """Motor allocation: per-rotor thrusts f = alloc [T, tau_x, tau_y, tau_z],
    clamped to [0, f_max], turned into rotor-speed commands on the thrust curve.
    It is also the torque interface of the first-principles model (command =
    collective thrust and body torques)."""
    A = P["alloc"].reshape(4, 4, -1)
    f = (A * wrench[None, :, :]).sum(1)
    f = torch.clamp(f, min=torch.zeros_like(f), max=P["f_max"][0:1].expand_as(f))
    return rotor_speed_for_thrust(f, P)


# ---- identified model -----------------------------------------------------------

def id_rates(x: torch.Tensor, u: torch.Tensor, P) -> torch.Tensor:
    """Time derivative of the 13-component identified state [p, Psi, v, dPsi, f]
    under u = [Psi_cmd, f_cmd] (Eqs. 3_simplified_*): p' = v;
    m v' = -m g e_z + R(Psi) e_z c_f f; f' = c_tau (f_cmd - f);
    Psi'' = c1 Psi + c2 Psi' + c3 Psi_cmd (per axis; reading of the garbled
    coefficient labels as three distinct 3-vectors); the drag term R f_a with
    f_a = C_a R^T v as in the first-principles model.

    The simplified variant without thrust dynamics (same section, last
    sentence; drag is removed by C_a = 0) is selected per drone by c_tau = 0:
    the commanded thrust acts directly (f = f_cmd in the acceleration) and the
    thrust row has zero rate; ``step_id`` then stores the applied thrust in
    that row, so the dynamic state is the 12 components [p, Psi, v, dPsi]."""
    psi, v, dpsi, fs = x[3:6], x[6:9], x[9:12], x[12]
    m, g = P["mass"][0], P["gravity"][0]
    direct = P["c_tau"][0] == 0
    fs = torch.where(direct, u[3], fs)
    acc = (P["c_f"][0] * fs / m) * euler_zyx_body_z(psi)
    acc = acc - torch.stack([torch.zeros_like(g), torch.zeros_like(g), g])
    acc = acc + drag_acceleration(euler_zyx_matrix(psi), v, P)
    ddpsi = P["c_psi1"] * psi + P["c_psi2"] * dpsi + P["c_psi3"] * u[0:3]
    dfs = P["c_tau"][0] * (u[3] - fs)
    return torch.cat([v, dpsi, acc, ddpsi, dfs[None]], 0)


# ---- integration and the step ----------------------------------------------------

def integrate(rates, x: torch.Tensor, dt: float, integrator: int) -> torch.Tensor:
    """Explicit Euler, or classical four-stage RK4, with the command held."""
    if integrator == EULER:
        return x + dt * rates(x)
    k1 = rates(x)
    k2 = rates(x + (dt / 2) * k1)
    k3 = rates(x + (dt / 2) * k2)
    k4 = rates(x + dt * k3)
    return x + (dt / 6) * (k1 + 2 * k2 + 2 * k3 + k4)


def _advance_fp(x, rot_cmd, ctrl, P, integrator: int, dt: float, renorm: bool):
    """Integrate the 17 rigid-body and rotor components under rotor-speed commands
    held over the step, renormalise the quaternion, append the controller state."""
    body = integrate(lambda s: fp_rates(s, rot_cmd, P), x[0:17], dt, integrator)
    if renorm:
        q = body[3:7]
        body = torch.cat([body[0:3], q / torch.sqrt((q * q).sum(0)), body[7:17]], 0)
    if ctrl is None:
        return body
    return torch.cat([body, ctrl], 0)


def step_fp(x, u, P, control: int, integrator: int, dt: float, renorm: bool = True):
    """One step of a first-principles drone (state 17, or 25 with the PID)."""
    if control == CTRL_ATT_PID:
        rot_cmd, ctrl = attitude_pid(x, u, P, dt)
    elif control == CTRL_TORQUE:
        rot_cmd, ctrl = allocate(u, P), None
    elif control == CTRL_POSITION:
        rot_cmd, ctrl = position_controller(x, u, P), None
    else:
        rot_cmd, ctrl = u, None
    return _advance_fp(x, rot_cmd, ctrl, P, integrator, dt, renorm)


def step_fp_multirate(x, u, P, control: int, integrator: int, dt: float, renorm: bool,
                      run_ctrl: bool, held, dt_ctrl: float):
    """One physics step of a first-principles drone whose onboard controller runs
    at a lower rate than the physics (control interfaces and rates, section
    "Architecture"; reading: the controller is evaluated at the start of every
    block of n physics steps with its own period dt_ctrl = n dt, and its rotor
    commands are held, zero-order, until the next evaluation). On a controller
    step the attitude PID, position controller or torque allocation is evaluated
    and its rotor commands become the held ones; on the other steps the held
    commands drive the rotors and the controller state is carried unchanged. The
    rotor interface has no onboard controller: its commands apply every step.
    Returns (next state, held rotor commands)."""
    if control == CTRL_ROTOR:
        return step_fp(x, u, P, control, integrator, dt, renorm), None
    if run_ctrl:
        if control == CTRL_ATT_PID:
            rot_cmd, ctrl = attitude_pid(x, u, P, dt_ctrl)
        elif control == CTRL_TORQUE:
            rot_cmd, ctrl = allocate(u, P), None
        else:
            rot_cmd, ctrl = position_controller(x, u, P), None
    else:
        rot_cmd = held
        ctrl = x[17:25] if control == CTRL_ATT_PID else None
    return _advance_fp(x, rot_cmd, ctrl, P, integrator, dt, renorm), rot_cmd


def step_id(x, u, P, integrator: int, dt: float):
    y = integrate(lambda s: id_rates(s, u, P), x[0:13], dt, integrator)
    direct = P["c_tau"][0] == 0
    if bool(direct.any()):
        y = torch.cat([y[0:12], torch.where(direct, u[3], y[12])[None]], 0)
    return y


class Batch:
    """Per-drone view of a set of worlds (models, parameters, world index)."""

    def __init__(self, drones_per_world, model_per_world, params, control, integrator,
                 dt, renorm=1, ctrl_every=1):
        self.counts = np.asarray(drones_per_world, np.int64)
        self.models = np.asarray(model_per_world, np.int64)
        self.world = np.repeat(np.arange(len(self.counts)), self.counts)
        self.D = int(self.counts.sum())
        dm = self.models[self.world]
        self.fp_idx = torch.as_tensor(np.nonzero(dm == MODEL_FP)[0])
        self.id_idx = torch.as_tensor(np.nonzero(dm == MODEL_ID)[0])
        P = per_drone_params(params, self.counts)
        self.P_fp = {k: v[:, self.fp_idx] for k, v in P.items()}
        self.P_id = {k: v[:, self.id_idx] for k, v in P.items()}
        self.P = P
        self.control = int(control)
        self.integrator = int(integrator)
        self.dt = float(dt)
        self.renorm = bool(renorm)
        self.ctrl_every = max(int(ctrl_every), 1)

    @classmethod
    def from_workload(cls, w):
        return cls(w.drones_per_world, w.model_per_world, w.params, w.control,
                   w.integrator, w.dt, w.renorm_q, getattr(w, "ctrl_every", 1))

    def step(self, x: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
        """x ``[S, D]`` -> state after one step under command u ``[4, D]``."""
        out = x
        if len(self.fp_idx):
            xf = x[:, self.fp_idx]
            nf = 25 if self.control == CTRL_ATT_PID else 17
            yf = step_fp(xf[:nf], u[:, self.fp_idx], self.P_fp, self.control,
                         self.integrator, self.dt, self.renorm)
            if x.shape[0] > nf:
                yf = torch.cat([yf, xf[nf:]], 0)
            out = out.index_copy(1, self.fp_idx, yf)
        if len(self.id_idx):
            xi = x[:, self.id_idx]
            yi = step_id(xi[:13], u[:, self.id_idx], self.P_id, self.integrator, self.dt)
            if x.shape[0] > 13:
                yi = torch.cat([yi, xi[13:]], 0)
            out = out.index_copy(1, self.id_idx, yi)
        return out

    def step_at(self, x: torch.Tensor, u: torch.Tensor, n: int, held):
        """Physics step n of a run in which the first-principles drones' onboard
        controller runs on the steps with n % ctrl_every == 0 (period ctrl_every
        dt) and its rotor commands are held in between (``step_fp_multirate``).
        ``held`` carries those commands between calls (None before the first).
        Returns (next state, held). With ctrl_every = 1 this is ``step``."""
        if self.ctrl_every == 1 or len(self.fp_idx) == 0 or self.control == CTRL_ROTOR:
            return self.step(x, u), held
        out = x
        xf = x[:, self.fp_idx]
        nf = 25 if self.control == CTRL_ATT_PID else 17
        yf, held = step_fp_multirate(xf[:nf], u[:, self.fp_idx], self.P_fp, self.control, self.integrator,
                                     self.dt, self.renorm, n % self.ctrl_every == 0, held,
                                     self.ctrl_every * self.dt)
        if x.shape[0] > nf:
            yf = torch.cat([yf, xf[nf:]], 0)
        out = out.index_copy(1, self.fp_idx, yf)
        if len(self.id_idx):
            xi = x[:, self.id_idx]
            yi = step_id(xi[:13], u[:, self.id_idx], self.P_id, self.integrator, self.dt)
            if x.shape[0] > 13:
                yi = torch.cat([yi, xi[13:]], 0)
            out = out.index_copy(1, self.id_idx, yi)
        return out, held

    # -- reference and objective -------------------------------------------------

    def figure_eight(self, t: float, amp: float, period: float, offset, shift=None):
        """Lemniscate of Gerono: p = [A sin(2 pi t/P), (A/2) sin(4 pi t/P), 0] plus
        the drone's offset; returns (p_ref [3,D], v_ref [3,D]). With ``shift`` [D]
        (seconds) drone d is evaluated at t + shift_d instead."""
        w0 = 2 * math.pi / period
        if shift is not None:
            td = t + t64(shift)
            z = torch.zeros(self.D, dtype=F64)
            p = torch.stack([amp * torch.sin(w0 * td), 0.5 * amp * torch.sin(2 * w0 * td), z])
            v = torch.stack([amp * w0 * torch.cos(w0 * td), amp * w0 * torch.cos(2 * w0 * td), z])
            return (p + offset if offset is not None else p), v
        p = torch.tensor([amp * math.sin(w0 * t), 0.5 * amp * math.sin(2 * w0 * t), 0.0], dtype=F64)
        v = torch.tensor([amp * w0 * math.cos(w0 * t), amp * w0 * math.cos(2 * w0 * t), 0.0], dtype=F64)
        p = p[:, None].expand(3, self.D)
        if offset is not None:
            p = p + offset
        return p, v[:, None].expand(3, self.D)

    def reference_state(self, p_ref, v_ref):
        """The 13-component reference the feedback compares against: first-principles
        [p_ref, (0,0,0,1), v_ref, 0]; identified [p_ref, 0, v_ref, 0, m g / c_f]."""
        xr = torch.zeros(13, self.D, dtype=F64)
        xr[0:3] = p_ref
        if len(self.fp_idx):
            f = self.fp_idx
            xr[6, f] = 1.0
            xr[7:10, f] = v_ref[:, f]
        if len(self.id_idx):
            i = self.id_idx
            xr[6:9, i] = v_ref[:, i]
            xr[12, i] = self.P_id["mass"][0] * self.P_id["gravity"][0] / self.P_id["c_f"][0]
        return xr


def _safe_sqrt(a: torch.Tensor) -> torch.Tensor:
    """sqrt with gradient 0 at 0 (a subgradient of the norm's kink)."""
    pos = a > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, a, torch.ones_like(a))), torch.zeros_like(a))


def tilt_angle(batch: "Batch", x: torch.Tensor) -> torch.Tensor:
    """Angle between the body z axis and the world z axis (the reward's angle
    from the upright orientation): first principles 2 asin(|(q_x, q_y)| / |q|);
    identified atan2(sqrt(sin^2 phi + cos^2 phi sin^2 theta), cos phi cos theta)
    (the same angle for R = Rz Ry Rx, written without cancellation)."""
    out = torch.zeros(batch.D, dtype=x.dtype)
    if len(batch.fp_idx):
        q = x[3:7, batch.fp_idx]
        s2 = (q[0] * q[0] + q[1] * q[1]) / (q * q).sum(0)
        out = out.index_copy(0, batch.fp_idx, 2 * torch.asin(torch.clamp(_safe_sqrt(s2), max=1.0)))
    if len(batch.id_idx):
        phi, th = x[3, batch.id_idx], x[4, batch.id_idx]
        a = torch.sin(phi) ** 2 + (torch.cos(phi) * torch.sin(th)) ** 2
        out = out.index_copy(0, batch.id_idx, torch.atan2(_safe_sqrt(a), torch.cos(phi) * torch.cos(th)))
    return out


def hover_action(batch: "Batch") -> torch.Tensor:
    """The commands that hold a drone in hover, per drone ``[4, D]``: identified
    [0, 0, 0, m g / c_f]; attitude interface [0, 0, 0, m g]; torque interface
    [m g, 0, 0, 0]; rotor interface the hover speed on every rotor. The position
    interface has none (its command is a place, not an action)."""
    a = torch.zeros(4, batch.D, dtype=F64)
    if len(batch.fp_idx):
        P = batch.P_fp
        mg = P["mass"][0] * P["gravity"][0]
        if batch.control == CTRL_ATT_PID:
            a[3, batch.fp_idx] = mg
        elif batch.control == CTRL_TORQUE:
            a[0, batch.fp_idx] = mg
        elif batch.control == CTRL_ROTOR:
            a[:, batch.fp_idx] = rotor_speed_for_thrust(0.25 * mg[None, :].expand(4, -1), P)
        else:
            raise ValueError("the position interface has no hover action")
    if len(batch.id_idx):
        P = batch.P_id
        a[3, batch.id_idx] = P["mass"][0] * P["gravity"][0] / P["c_f"][0]
    return a


def mlp_param_count(hidden: int) -> int:
    """Parameters of the small MLP policy with `hidden` units per hidden layer."""
    H = int(hidden)
    return 13 * H + H + H * H + H + 4 * H + 4


def mlp_policy(theta: torch.Tensor, hidden: int, e: torch.Tensor) -> torch.Tensor:
    """Small MLP actor of the BPTT setup (Methods, "Backpropagation Through Time":
    an actor network trained on analytical gradients; its architecture is not
    printed). Reading: o = W3 tanh(W2 tanh(W1 e + b1) + b2) + b3 on the tracking
    error e [13, D], tanh hidden layers of `hidden` units, linear output [4, D].
    theta [D, P] holds each drone's parameters, packed
    [W1 (H x 13, row-major) | b1 (H) | W2 (H x H) | b2 (H) | W3 (4 x H) | b3 (4)]."""
    H = int(hidden)
    D = theta.shape[0]
    o = 0
    W1 = theta[:, o:o + 13 * H].reshape(D, H, 13); o += 13 * H
    b1 = theta[:, o:o + H]; o += H
    W2 = theta[:, o:o + H * H].reshape(D, H, H); o += H * H
    b2 = theta[:, o:o + H]; o += H
    W3 = theta[:, o:o + 4 * H].reshape(D, 4, H); o += 4 * H
    b3 = theta[:, o:o + 4]
    h1 = torch.tanh(torch.einsum("dji,di->dj", W1, e.T) + b1)
    h2 = torch.tanh(torch.einsum("djk,dk->dj", W2, h1) + b2)
    return (torch.einsum("dok,dk->do", W3, h2) + b3).T


def rollout(batch: Batch, x0: torch.Tensor, cmds: torch.Tensor, steps: int,
            gain: Optional[torch.Tensor] = None, gain_index=None,
            ref_amp: float = 1.0, ref_period: float = 4.0, ref_offset=None,
            ref_table: Optional[torch.Tensor] = None, w_u: float = 1e-3,
            with_loss: bool = True, keep_traj: bool = False, reward: Optional[Dict] = None,
            policy_hidden: int = 0, ref_step0: int = 0, ref_time_shift=None, policy_scale=None):
    """Roll out ``steps`` steps with per-step commands ``cmds`` [T, 4, D] (or held
    [4, D]). With ``gain`` [G, 4, 13] the applied command is
    u_t = ubar_t + G_w (x_t[0:13] - x_ref(t)). Loss per drone:
    sum_{t=1..T} |p_t - p_ref(t)|^2 + w_u sum_{t=0..T-1} |u_t|^2, with t_n = n dt.

    With ``reward`` = dict(w_tilt, w_act[4], w_dact[4]) the loss is instead minus
    the summed reward of the paper's BPTT tracking task (Methods,
    "Backpropagation Through Time"): for t = 0..T-1, with the action a_t = u_t
    and the state x_{t+1} it leads to,
      r_t = exp(-2 |p_{t+1} - p_ref(t+1)|) - w_tilt * tilt(x_{t+1})
            - sum_i w_act_i (a_t,i - a_hover,i)^2 - sum_i w_dact_i (a_t,i - a_{t-1},i)^2
    (reading: the previous action before the first step is the hover action;
    the goal is the reference point; norms have gradient 0 at their kink).

    With ``policy_hidden`` = H > 0, ``gain`` [G, P] holds MLP policies instead of
    linear gains and u_t = ubar_t + mlp_policy(theta_w, H, x_t[0:13] - x_ref(t)). With
    ``ref_step0`` = k the figure-eight is followed from t = k dt: step n tracks
    p_ref((k + n) dt), so that consecutive rollouts continue along it. With
    ``ref_time_shift`` [D] drone d follows the figure-eight at t + shift_d
    (starts spread along the trajectory; not with ``ref_table``). With
    ``policy_scale`` s (4 values, not all 0) the policy output o (linear or MLP)
    enters as s * tanh(o): a normalised action in [-1, 1] mapped linearly onto
    each command's range.
    Returns dict(x=x_T, loss=[D] or None, traj=[T+1, S, D] or None)."""
    x = x0
    D = batch.D
    G = None
    if gain is not None:
        gi = np.zeros(len(batch.counts), np.int64) if gain_index is None else np.asarray(gain_index, np.int64)
        G = gain[torch.as_tensor(gi[batch.world])]            # [D, 4, 13], or [D, P] for an MLP policy
    loss = torch.zeros(D, dtype=F64)
    traj = [x] if keep_traj else None
    if ref_time_shift is not None and ref_table is not None:
        raise ValueError("a time shift applies to the figure-eight only")
    squash = None
    if policy_scale is not None and any(float(v) != 0.0 for v in policy_scale):
        squash = t64(np.asarray(policy_scale, np.float32))[:, None]

    def ref(n):
        t = (ref_step0 + n) * batch.dt
        if ref_table is not None:
            xr = ref_table[n][:, None].expand(13, D)
            if ref_offset is not None:
                xr = torch.cat([xr[0:3] + ref_offset, xr[3:]], 0)
            return xr[0:3], xr
        p, v = batch.figure_eight(t, ref_amp, ref_period, ref_offset, ref_time_shift)
        return p, (batch.reference_state(p, v) if G is not None else None)

    held = None
    if reward is not None:
        a_hover = hover_action(batch)
        w_act = t64(reward["w_act"])[:, None]
        w_dact = t64(reward["w_dact"])[:, None]
        u_prev = a_hover
    for n in range(steps):
        ubar = cmds[n] if cmds.dim() == 3 else cmds
        if G is not None:
            _, xr = ref(n)
            e = x[0:13] - xr
            if policy_hidden:
                o = mlp_policy(G, policy_hidden, e)
            else:
                o = (G * e.T[:, None, :]).sum(2).T
            if squash is not None:
                o = squash * torch.tanh(o)
            u = ubar + o
        else:
            u = ubar
        if with_loss and reward is None:
            loss = loss + w_u * (u * u).sum(0)
        x, held = batch.step_at(x, u, n, held)
        if with_loss:
            p_ref, _ = ref(n + 1)
            d = x[0:3] - p_ref
            if reward is None:
                loss = loss + (d * d).sum(0)
            else:
                r = (torch.exp(-2 * _safe_sqrt((d * d).sum(0))) - reward["w_tilt"] * tilt_angle(batch, x)
                     - (w_act * (u - a_hover) ** 2).sum(0) - (w_dact * (u - u_prev) ** 2).sum(0))
                loss = loss - r
                u_prev = u
        if keep_traj:
            traj.append(x)
    return {"x": x, "loss": loss if with_loss else None,
            "traj": torch.stack(traj) if keep_traj else None}


def rollout_grad(batch: Batch, x0, cmds, steps, gain=None, gain_index=None, dloss=None, **kw):
    """Exact reverse-mode gradient of sum_d dloss_d * loss_d with respect to the
    per-step commands, the initial state and the gain (autograd on the FP64 map)."""
    x0 = t64(x0).clone().requires_grad_(True)
    cmds = t64(cmds).clone().requires_grad_(True)
    leaves = [x0, cmds]
    if gain is not None:
        gain = t64(gain).clone().requires_grad_(True)
        leaves.append(gain)
    out = rollout(batch, x0, cmds, steps, gain=gain, gain_index=gain_index, **kw)
    seed = torch.ones(batch.D, dtype=F64) if dloss is None else t64(dloss)
    total = (seed * out["loss"]).sum()
    grads = torch.autograd.grad(total, leaves, allow_unused=True)
    res = {"loss": out["loss"].detach(), "x": out["x"].detach(),
           "g_x0": grads[0], "g_cmds": grads[1]}
    if gain is not None:
        res["g_gain"] = grads[2]
    return res


# ---- convenience entry points on a workload --------------------------------------

def simulate_held(w, steps: Optional[int] = None, x0=None, store_every: Optional[int] = None) -> torch.Tensor:
    """State after ``steps`` steps with the workload's held command ``[4, D]``.

    ``store_every = k`` rounds the state to binary32 after every k steps: the
    state a caller sees who keeps it in the public binary32 layout between
    calls of k steps each (the steps themselves stay in fp64). This models the
    storage format only, not any kernel's arithmetic."""
    b = Batch.from_workload(w)
    x = t64(w.x0 if x0 is None else x0)
    u = t64(w.cmds)
    n = w.steps if steps is None else steps
    held = None
    with torch.no_grad():
        for i in range(n):
            x, held = b.step_at(x, u, i, held)
            if store_every and (i + 1) % store_every == 0:
                x = x.to(torch.float32).to(torch.float64)
    return x


def rollout_workload(w, with_grad: bool = False, keep_traj: bool = False):
    b = Batch.from_workload(w)
    kw = dict(ref_amp=w.ref_amp, ref_period=w.ref_period,
              ref_offset=None if w.ref_offset is None else t64(w.ref_offset), w_u=w.w_u,
              reward=getattr(w, "reward", None), policy_hidden=getattr(w, "policy_hidden", 0),
              ref_step0=getattr(w, "ref_step0", 0),
              ref_time_shift=getattr(w, "ref_time_shift", None),
              policy_scale=getattr(w, "policy_scale", None))
    gain = None if w.gain is None else t64(w.gain)
    if with_grad:
        return rollout_grad(b, w.x0, w.cmds, w.steps, gain=gain, gain_index=w.gain_index,
                            dloss=w.dloss, **kw)
    with torch.no_grad():
        return rollout(b, t64(w.x0), t64(w.cmds), w.steps, gain=gain,
                       gain_index=w.gain_index, keep_traj=keep_traj, **kw)
