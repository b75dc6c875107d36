"""Seeded synthetic workloads for the batched drone step.

This module only draws random numbers and lays them out. It contains none of the
simulation arithmetic (no derivative, controller, integrator or loss); both the
FP64 oracle and the GPU path consume what it returns.

Every array is rounded to float32 before it is handed out, so both sides start
from the same FP32 values (the oracle promotes them to FP64).

Shapes follow the structure-of-arrays convention of the C interface:
state ``[S][D]``, held commands ``[4][D]``, per-step commands ``[T][4][D]``,
per-world parameters as named ``[M, k]`` arrays. ``D`` is the total drone count,
worlds are concatenated in world order.

Random streams are ``numpy.random.Generator(numpy.random.Philox(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

# ---- enum values of the C interface (include/cfsim.h) -----------------------
MODEL_FP = 0          # first-principles rigid body + rotor dynamics
MODEL_ID = 1          # identified (abstracted) attitude-command model
CTRL_ROTOR = 0        # first-principles worlds take rotor-speed commands
CTRL_ATT_PID = 1      # first-principles worlds take [roll, pitch, yaw-rate, thrust]
CTRL_TORQUE = 2       # first-principles worlds take [thrust, tau_x, tau_y, tau_z]
CTRL_POSITION = 3     # first-principles worlds take [x, y, z, yaw] setpoints
INTEG_EULER = 0
INTEG_RK4 = 1

S_FP_ROTOR = 17       # p(3) q(4, scalar last) v(3) w_body(3) Omega(4)
S_FP_PID = 25         # + angle integrals(2) rate integrals(3) previous body rate(3)
S_ID = 13             # p(3) Psi(3) v(3) dPsi(3) f_sum(1)

# Named per-world parameter fields and their widths, in record order.
PARAM_FIELDS = (
    ("mass", 1), ("gravity", 1), ("J", 3),
    ("thrust_poly", 3), ("torque_poly", 3),
    ("mix_tx", 4), ("mix_ty", 4), ("mix_yaw", 4),
    ("motor_up", 2), ("motor_down", 2),
    ("Jp", 1), ("drag", 3),
    ("ang_kp", 2), ("ang_ki", 2), ("rate_kp", 3), ("rate_ki", 3), ("rate_kd", 3),
    ("J_ctrl", 3), ("f_max", 1), ("alloc", 16),
    ("c_f", 1), ("c_tau", 1), ("c_psi1", 3), ("c_psi2", 3), ("c_psi3", 3),
    ("pos_kp", 3), ("pos_kv", 3), ("att_kr", 3), ("att_kw", 3),
)

# ---- nominal Crazyflie-class airframe (synthetic values) --------------------
MASS = 0.027
GRAVITY = 9.81
INERTIA = (1.4e-5, 1.4e-5, 2.2e-5)
K_THRUST = 3e-10            # f = K_THRUST * Omega^2
TORQUE_RATIO = 0.006        # rotor drag torque = TORQUE_RATIO * f
ARM = 0.046                 # motor distance from the centre
MOTOR_TAU = 0.03            # rotor-speed time constant [s]
THRUST_TO_WEIGHT = 1.9
# attitude PID gains (own design, normalised by the nominal inertia)
ANG_KP, ANG_KI = 6.0, 1.0
RATE_KP, RATE_KI, RATE_KD = 17.0, 5.0, 0.1
# geometric position controller (position interface), per axis
POS_KP = (4.0, 4.0, 6.0)     # [1/s^2]
POS_KV = (4.0, 4.0, 5.0)     # [1/s]
ATT_KR = (100.0, 100.0, 25.0)  # [1/s^2]
ATT_KW = (20.0, 20.0, 10.0)    # [1/s]
# identified model nominal response
ID_TAU = (0.06, 0.06, 0.12)
ID_GAIN = (1.0, 1.0, 1.0)
ID_CF = 1.0
ID_CTAU = 1.0 / 0.03


@dataclasses.dataclass
class Workload:
    name: str
    n_worlds: int
    drones_per_world: np.ndarray          # int32 [M]
    model_per_world: np.ndarray           # uint8 [M]
    control: int
    integrator: int
    dt: float
    renorm_q: int
    params: Dict[str, np.ndarray]         # name -> float32 [M, k]
    x0: np.ndarray                        # float32 [S, D]
    steps: int
    cmds: np.ndarray                      # float32 [4, D] (held) or [T, 4, D]
    gain: Optional[np.ndarray] = None     # float32 [G, 4, 13]
    gain_index: Optional[np.ndarray] = None   # int32 [M]
    ref_amp: float = 1.0
    ref_period: float = 4.0
    ref_offset: Optional[np.ndarray] = None   # float32 [3, D]
    w_u: float = 1e-3
    dloss: Optional[np.ndarray] = None    # float32 [D]
    ctrl_every: int = 1                   # onboard controller every n physics steps
    reward: Optional[dict] = None         # BPTT reward weights (w_tilt, w_act[4], w_dact[4]) or None
    policy_hidden: int = 0                # > 0: `gain` holds [G, P] small-MLP policies of this width
    ref_step0: int = 0                    # the figure-eight is followed from t = ref_step0 dt
    ref_time_shift: Optional[np.ndarray] = None   # float32 [D]: drone d follows it at t + shift_d
    policy_scale: Optional[np.ndarray] = None     # float32 [4]: policy output o enters as s * tanh(o)

    @property
    def n_drones_total(self) -> int:
        return int(self.drones_per_world.sum())

    @property
    def state_dim(self) -> int:
        return int(self.x0.shape[0])

    def world_offsets(self) -> np.ndarray:
        off = np.zeros(self.n_worlds + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.drones_per_world)
        return off


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def empty_params(n_worlds: int) -> Dict[str, np.ndarray]:
    return {name: np.zeros((n_worlds, k), dtype=np.float64) for name, k in PARAM_FIELDS}


def fill_fp_airframe(P: Dict[str, np.ndarray], worlds, mass, inertia) -> None:
    """Crazyflie-class first-principles parameters for the given worlds.

    ``mass`` [n], ``inertia`` [n, 3] are the (possibly perturbed) physical values;
    the controller keeps the nominal inertia and motor limits.
    """
    worlds = np.asarray(worlds)
    a = ARM / math.sqrt(2.0)
    P["mass"][worlds, 0] = mass
    P["gravity"][worlds, 0] = GRAVITY
    P["J"][worlds] = inertia
    P["thrust_poly"][worlds] = (0.0, 0.0, K_THRUST)
    P["torque_poly"][worlds] = (0.0, 0.0, TORQUE_RATIO * K_THRUST)
    # motors 1..4 at (+a,-a), (-a,-a), (-a,+a), (+a,+a); yaw reaction signs -,+,-,+
    P["mix_tx"][worlds] = (-a, -a, a, a)
    P["mix_ty"][worlds] = (-a, a, a, -a)
    P["mix_yaw"][worlds] = (-1.0, 1.0, -1.0, 1.0)
    P["motor_up"][worlds] = (1.0 / MOTOR_TAU, 0.0)
    P["motor_down"][worlds] = (1.0 / MOTOR_TAU, 0.0)
    P["ang_kp"][worlds] = ANG_KP
    P["ang_ki"][worlds] = ANG_KI
    P["rate_kp"][worlds] = RATE_KP
    P["rate_ki"][worlds] = RATE_KI
    P["rate_kd"][worlds] = RATE_KD
    P["J_ctrl"][worlds] = INERTIA
    P["f_max"][worlds, 0] = THRUST_TO_WEIGHT * MASS * GRAVITY / 4.0
    P["pos_kp"][worlds] = POS_KP
    P["pos_kv"][worlds] = POS_KV
    P["att_kr"][worlds] = ATT_KR
    P["att_kw"][worlds] = ATT_KW
    # Allocation (controller mixer) of the x airframe: per-motor thrust from
    # [collective thrust, tau_x, tau_y, tau_z]; row i = motor i.
    sx = (-1.0, -1.0, 1.0, 1.0)
    sy = (-1.0, 1.0, 1.0, -1.0)
    sz = (-1.0, 1.0, -1.0, 1.0)
    alloc = np.zeros((4, 4))
    for i in range(4):
        alloc[i] = (0.25, sx[i] / (4 * a), sy[i] / (4 * a), sz[i] / (4 * TORQUE_RATIO))
    P["alloc"][worlds] = alloc.reshape(16)


def fill_id_model(P: Dict[str, np.ndarray], worlds, gain, tau) -> None:
    """Identified attitude model with a critically damped second-order response
    per axis: DC gain ``gain`` [n,3] and time constant ``tau`` [n,3]."""
    worlds = np.asarray(worlds)
    P["mass"][worlds, 0] = MASS
    P["gravity"][worlds, 0] = GRAVITY
    P["c_f"][worlds, 0] = ID_CF
    P["c_tau"][worlds, 0] = ID_CTAU
    P["c_psi1"][worlds] = -1.0 / tau ** 2
    P["c_psi2"][worlds] = -2.0 / tau
    P["c_psi3"][worlds] = gain / tau ** 2


def hover_speed(mass) -> np.ndarray:
    return np.sqrt(np.asarray(mass) * GRAVITY / (4.0 * K_THRUST))


def _finish_params(P) -> Dict[str, np.ndarray]:
    return {k: _f32(v) for k, v in P.items()}


def _random_attitude(rng, n, max_angle):
    axis = rng.normal(size=(3, n))
    axis /= np.linalg.norm(axis, axis=0, keepdims=True)
    ang = rng.uniform(0.0, max_angle, size=n)
    return np.concatenate([axis * np.sin(ang / 2), np.cos(ang / 2)[None]], axis=0)


def _grid_positions(rng, n, dims=None, spacing=0.3, jitter=0.03):
    """First ``n`` points of a jittered grid. ``dims`` = (nx, ny, nz) or a cube."""
    if dims is None:
        side = max(1, int(math.ceil(round(n ** (1.0 / 3.0), 9))))
        while side ** 3 < n:
            side += 1
        dims = (side, side, side)
    nx, ny, nz = dims
    idx = np.arange(n)
    ix, iy, iz = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    pos = np.stack([ix, iy, iz]).astype(np.float64) * spacing
    pos += rng.uniform(-jitter, jitter, size=(3, n))
    return pos


# ---- the five workloads ------------------------------------------------------

def fp_rotor_open_loop(seed: int = 1001, n_worlds: int = 16, steps: int = 500,
            integrator: int = INTEG_RK4, dt: float = 0.002) -> Workload:
    """Plain forward, first-principles rotor-speed interface, 1 drone per world."""
    rng = _rng(seed)
    M = D = n_worlds
    P = empty_params(M)
    fill_fp_airframe(P, np.arange(M), np.full(M, MASS), np.tile(INERTIA, (M, 1)))
    wh = hover_speed(MASS)
    x0 = np.zeros((S_FP_ROTOR, D))
    x0[0:3] = rng.uniform(-1.0, 1.0, size=(3, D))
    x0[7:10] = rng.normal(0.0, 0.1, size=(3, D))
    x0[3:7] = _random_attitude(rng, D, 0.3)
    x0[13:17] = wh
    cmds = wh * (1.0 + 0.05 * rng.normal(size=(steps, 4, D)))
    return Workload("fp_rotor_open_loop", M, np.ones(M, np.int32),
                    np.full(M, MODEL_FP, np.uint8), CTRL_ROTOR, integrator,
                    float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(cmds))


def fp_torque(seed: int = 1006, n_worlds: int = 256, steps: int = 250, dt: float = 0.004) -> Workload:
    """Torque interface of the first-principles model (collective thrust and body
    torques at 250 Hz, 1 s open loop): per-world mass and inertia x U[0.9, 1.1],
    held commands thrust ~ m g U[0.9, 1.1], torques ~ N(0, (2e-5 N m)^2)."""
    rng = _rng(seed)
    M = D = n_worlds
    P = empty_params(M)
    mass = MASS * rng.uniform(0.9, 1.1, size=M)
    inertia = np.asarray(INERTIA)[None, :] * rng.uniform(0.9, 1.1, size=(M, 3))
    fill_fp_airframe(P, np.arange(M), mass, inertia)
    x0 = np.zeros((S_FP_ROTOR, D))
    x0[0:3] = rng.uniform(-1.0, 1.0, size=(3, D))
    x0[3:7] = _random_attitude(rng, D, 0.2)
    x0[13:17] = hover_speed(mass)
    cmds = np.empty((4, D))
    cmds[0] = mass * GRAVITY * rng.uniform(0.9, 1.1, size=D)
    cmds[1:4] = rng.normal(0.0, 2e-5, size=(3, D))
    return Workload("fp_torque_interface", M, np.ones(M, np.int32), np.full(M, MODEL_FP, np.uint8),
                    CTRL_TORQUE, INTEG_RK4, float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps,
                    _f32(cmds))


def fp_position(seed: int = 1010, n_worlds: int = 256, steps: int = 500, dt: float = 0.002) -> Workload:
    """Position interface of the first-principles model (geometric controller):
    per-world mass and inertia x U[0.9, 1.1], start at rest at p ~ U[-1, 1]^3 with
    hover rotors, held setpoints p + U[-1, 1]^3 and yaw ~ U[-0.5, 0.5] rad."""
    rng = _rng(seed)
    M = D = n_worlds
    P = empty_params(M)
    mass = MASS * rng.uniform(0.9, 1.1, size=M)
    inertia = np.asarray(INERTIA)[None, :] * rng.uniform(0.9, 1.1, size=(M, 3))
    fill_fp_airframe(P, np.arange(M), mass, inertia)
    x0 = np.zeros((S_FP_ROTOR, D))
    x0[0:3] = rng.uniform(-1.0, 1.0, size=(3, D))
    x0[6] = 1.0
    x0[13:17] = hover_speed(mass)
    cmds = np.empty((4, D))
    cmds[0:3] = x0[0:3] + rng.uniform(-1.0, 1.0, size=(3, D))
    cmds[3] = rng.uniform(-0.5, 0.5, size=D)
    return Workload("fp_position_interface", M, np.ones(M, np.int32), np.full(M, MODEL_FP, np.uint8),
                    CTRL_POSITION, INTEG_RK4, float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps,
                    _f32(cmds))


def _fp_pid_x0(D, mass_per_drone, pos=None):
    x0 = np.zeros((S_FP_PID, D))
    if pos is not None:
        x0[0:3] = pos
    x0[6] = 1.0
    x0[13:17] = hover_speed(mass_per_drone)
    return x0


def _attitude_cmds(rng, D):
    c = np.empty((4, D))
    c[0:2] = rng.uniform(-0.3, 0.3, size=(2, D))
    c[2] = rng.uniform(-0.3, 0.3, size=D)
    c[3] = rng.uniform(0.2, 0.5, size=D)
    return c


def fp_pid_closed_loop(seed: int = 1002, n_worlds: int = 4096, steps: int = 1000,
            dt: float = 0.002) -> Workload:
    """Closed loop: attitude commands -> cascaded PID -> mixer -> first-principles model."""
    rng = _rng(seed)
    M = D = n_worlds
    P = empty_params(M)
    mass = MASS * rng.uniform(0.9, 1.1, size=M)
    inertia = np.asarray(INERTIA)[None, :] * rng.uniform(0.9, 1.1, size=(M, 3))
    fill_fp_airframe(P, np.arange(M), mass, inertia)
    cmds = _attitude_cmds(rng, D)
    x0 = _fp_pid_x0(D, mass)
    return Workload("fp_pid_closed_loop", M, np.ones(M, np.int32),
                    np.full(M, MODEL_FP, np.uint8), CTRL_ATT_PID, INTEG_RK4,
                    float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(cmds))


def _id_world_response(rng, n):
    gain = np.asarray(ID_GAIN)[None, :] * rng.uniform(0.8, 1.2, size=(n, 3))
    tau = np.asarray(ID_TAU)[None, :] * rng.uniform(0.8, 1.2, size=(n, 3))
    return gain, tau


def _id_cmds(rng, D):
    c = np.empty((4, D))
    c[0:3] = rng.uniform(-0.1, 0.1, size=(3, D))
    c[3] = (MASS * GRAVITY / ID_CF) * rng.uniform(0.95, 1.05, size=D)
    return c


def _id_x0(D, pos):
    x0 = np.zeros((S_ID, D))
    x0[0:3] = pos
    x0[12] = MASS * GRAVITY / ID_CF
    return x0


def id_swarm(seed: int = 1003, n_worlds: int = 64, n_drones: int = 4000,
            steps: int = 1000, dt: float = 0.002, integrator: int = INTEG_RK4) -> Workload:
    """Swarm: identified attitude-command model, jittered 20x20x10 grid per world."""
    rng = _rng(seed)
    M, N = n_worlds, n_drones
    D = M * N
    P = empty_params(M)
    gain, tau = _id_world_response(rng, M)
    fill_id_model(P, np.arange(M), gain, tau)
    dims = (20, 20, 10) if N <= 4000 else None
    pos = np.concatenate([_grid_positions(rng, N, dims) for _ in range(M)], axis=1)
    x0 = _id_x0(D, pos)
    cmds = _id_cmds(rng, D)
    return Workload("id_swarm", M, np.full(M, N, np.int32),
                    np.full(M, MODEL_ID, np.uint8), CTRL_ATT_PID, integrator,
                    float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(cmds))


# weights of the paper's BPTT tracking reward (Methods, BPTT parameter table)
BPTT_REWARD = {"w_tilt": 0.1, "w_act": [0.12, 0.12, 0.0, 0.02], "w_dact": [1.4, 1.4, 0.0, 0.8]}


def id_rollout_grad(seed: int = 1004, n_worlds: int = 1024, steps: int = 500,
            dt: float = 0.002, gain_std: float = 0.01) -> Workload:
    """Differentiable rollout of the identified model with a shared 4x13 feedback gain,
    tracking a figure-eight (amplitude 1 m, period 4 s)."""
    rng = _rng(seed)
    M = D = n_worlds
    P = empty_params(M)
    fill_id_model(P, np.arange(M), np.tile(ID_GAIN, (M, 1)), np.tile(ID_TAU, (M, 1)))
    f_hover = MASS * GRAVITY / ID_CF
    x0 = _id_x0(D, rng.normal(0.0, 0.05, size=(3, D)))
    # velocity of the figure-eight at t = 0 is (2*pi*A/P, 2*pi*A/P, 0) = (pi/2, pi/2, 0)
    x0[6:9] = np.array([math.pi / 2, math.pi / 2, 0.0])[:, None] + rng.normal(0.0, 0.05, size=(3, D))
    ubar = np.zeros((steps, 4, D))
    ubar[:, 3] = f_hover
    ubar += rng.normal(0.0, 0.02, size=ubar.shape)
    gain = rng.normal(0.0, gain_std, size=(1, 4, 13))
    return Workload("id_rollout_grad", M, np.ones(M, np.int32),
                    np.full(M, MODEL_ID, np.uint8), CTRL_ATT_PID, INTEG_RK4,
                    float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(ubar),
                    gain=_f32(gain), gain_index=None, ref_amp=1.0, ref_period=4.0,
                    ref_offset=None, w_u=1e-3, dloss=np.ones(D, np.float32))


def gradient_goal(seed: int = 1007, n_worlds: int = 1 << 20, steps: int = 10,
                  dt: float = 0.002) -> Workload:
    """Gradient throughput workload: many single-drone worlds of the closed-loop
    first-principles model (config-2 distributions), a short horizon of per-step
    attitude commands, loss = distance to a per-drone goal at every step (a
    figure-eight of amplitude 0 centred on the goal) + 1e-3 |u|^2."""
    rng = _rng(seed)
    M = D = n_worlds
    P = empty_params(M)
    mass = MASS * rng.uniform(0.9, 1.1, size=M)
    inertia = np.asarray(INERTIA)[None, :] * rng.uniform(0.9, 1.1, size=(M, 3))
    fill_fp_airframe(P, np.arange(M), mass, inertia)
    x0 = _fp_pid_x0(D, mass, rng.normal(0.0, 0.05, size=(3, D)))
    cmds = np.empty((steps, 4, D))
    cmds[:, 0:3] = rng.uniform(-0.2, 0.2, size=(steps, 3, D))
    cmds[:, 3] = (mass * GRAVITY)[None, :] * rng.uniform(0.8, 1.2, size=(steps, D))
    goal = rng.uniform(-1.0, 1.0, size=(3, D))
    return Workload("fp_pid_goal_gradient", M, np.ones(M, np.int32),
                    np.full(M, MODEL_FP, np.uint8), CTRL_ATT_PID, INTEG_RK4,
                    float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(cmds),
                    gain=None, gain_index=None, ref_amp=0.0, ref_period=4.0,
                    ref_offset=_f32(goal), w_u=1e-3, dloss=np.ones(D, np.float32))


def mppi_task(seed: int = 1008, n_controllers: int = 5, n_samples: int = 100_000, horizon: int = 25,
              dt: float = 0.02, model: int = MODEL_FP, n_obstacles: int = 8, substeps: int = 1):
    """Sampled-rollout control task: one drone hovering at (-2, 0, 1) must reach
    (2, 0, 1) through seeded spherical obstacles; ``n_controllers`` controllers of
    ``n_samples`` samples each over ``horizon`` steps of ``dt`` (50 Hz by
    default). Returns (single-drone workload, controller parameters, initial
    mean [C][H][4] = hover command)."""
    rng = _rng(seed)
    P = empty_params(1)
    if model == MODEL_FP:
        fill_fp_airframe(P, np.arange(1), np.array([MASS]), np.asarray(INERTIA)[None, :])
        x0 = _fp_pid_x0(1, np.array([MASS]), np.array([[-2.0], [0.0], [1.0]]))
        hover = np.array([0.0, 0.0, 0.0, MASS * GRAVITY])
        sigma = [0.15, 0.15, 0.3, 0.05]
        u_lo, u_hi = [-0.6, -0.6, -2.0, 0.0], [0.6, 0.6, 2.0, 0.5]
        r_u = [0.1, 0.1, 0.01, 1.0]
        control = CTRL_ATT_PID
    else:
        fill_id_model(P, np.arange(1), np.asarray(ID_GAIN)[None, :], np.asarray(ID_TAU)[None, :])
        x0 = _id_x0(1, np.array([[-2.0], [0.0], [1.0]]))
        hover = np.array([0.0, 0.0, 0.0, MASS * GRAVITY / ID_CF])
        sigma = [0.15, 0.15, 0.3, 0.05]
        u_lo, u_hi = [-0.6, -0.6, -3.2, 0.0], [0.6, 0.6, 3.2, 0.5]
        r_u = [0.1, 0.1, 0.01, 1.0]
        control = CTRL_ATT_PID
    obs = np.zeros((n_obstacles, 4))
    obs[:, 0] = rng.uniform(-1.0, 1.0, n_obstacles)
    obs[:, 1] = rng.uniform(-0.5, 0.5, n_obstacles)
    obs[:, 2] = rng.uniform(0.6, 1.4, n_obstacles)
    obs[:, 3] = rng.uniform(0.15, 0.35, n_obstacles)
    w = Workload("mppi_obstacles", 1, np.ones(1, np.int32), np.full(1, model, np.uint8), control, INTEG_RK4,
                 float(np.float32(dt)), 1, _finish_params(P), _f32(x0), horizon, _f32(np.tile(hover, (1, 1)).T))
    f = lambda a: [float(np.float32(v)) for v in a]
    params = {
        "n_controllers": n_controllers, "n_samples": n_samples, "horizon": horizon, "substeps": substeps,
        "n_elite": max(1, int(math.ceil(0.01 * n_samples))),
        "sigma": f(sigma), "beta": float(np.float32(0.8)), "lambda": 1.0,
        "u_lo": f(u_lo), "u_hi": f(u_hi), "u_ref": f(hover), "r_u": f(r_u),
        "goal": [2.0, 0.0, 1.0], "q_p": 1.0, "q_v": 0.1, "w_obs": 100.0,
        "obstacles": _f32(obs), "seed": int(rng.integers(0, 2 ** 63)),
    }
    mean0 = _f32(np.tile(hover, (n_controllers, horizon, 1)))
    return w, params, mean0


def hbm_sweep(model: int, n_drones: int, seed: int = 1009, dt: float = 0.002) -> Workload:
    """Bandwidth sweep: one world of ``n_drones`` drones with held commands, first
    principles at the rotor interface (config-1 distributions, attitude within
    0.3 rad drawn per drone as a small rotation vector) or the identified model
    (config-3 distributions); drawn directly in float32 so that 2^24 drones stay
    cheap to generate."""
    rng = _rng(seed)
    D = int(n_drones)
    P = empty_params(1)
    f32 = np.float32
    if model == MODEL_FP:
        fill_fp_airframe(P, np.arange(1), np.array([MASS]), np.asarray(INERTIA)[None, :])
        wh = f32(hover_speed(MASS))
        x0 = np.zeros((S_FP_ROTOR, D), f32)
        x0[0:3] = rng.uniform(-1.0, 1.0, size=(3, D)).astype(f32)
        x0[7:10] = rng.normal(0.0, 0.1, size=(3, D)).astype(f32)
        half = rng.uniform(-0.075, 0.075, size=(3, D)).astype(f32)     # half-angle components
        x0[3:6] = half
        x0[6] = np.sqrt(1.0 - (half.astype(np.float64) ** 2).sum(0)).astype(f32)
        x0[13:17] = wh
        cmds = (wh * (1.0 + 0.05 * rng.standard_normal(size=(4, D), dtype=f32))).astype(f32)
        ctrl = CTRL_ROTOR
    else:
        fill_id_model(P, np.arange(1), np.asarray(ID_GAIN)[None, :], np.asarray(ID_TAU)[None, :])
        x0 = np.zeros((S_ID, D), f32)
        x0[0:3] = rng.uniform(-3.0, 3.0, size=(3, D)).astype(f32)
        x0[12] = f32(MASS * GRAVITY / ID_CF)
        cmds = np.empty((4, D), f32)
        cmds[0:3] = rng.uniform(-0.1, 0.1, size=(3, D)).astype(f32)
        cmds[3] = (MASS * GRAVITY / ID_CF) * rng.uniform(0.95, 1.05, size=D).astype(f32)
        ctrl = CTRL_ATT_PID
    return Workload(f"hbm_sweep_{'fp' if model == MODEL_FP else 'id'}_{D}", 1, np.array([D], np.int32),
                    np.full(1, model, np.uint8), ctrl, INTEG_RK4, float(np.float32(dt)), 1,
                    _finish_params(P), x0, 100, cmds)


def uneven_counts(rng, n_worlds, n_max=4000):
    n = np.round(np.exp(rng.uniform(0.0, math.log(n_max), size=n_worlds)))
    return np.clip(n, 1, n_max).astype(np.int32)


def uneven_mixed(seed: int = 1005, n_worlds: int = 2048, steps: int = 1000, dt: float = 0.002,
            n_max: int = 4000) -> Workload:
    """Uneven batch: log-uniform drones per world, half first-principles closed loop,
    half identified model, held commands."""
    rng = _rng(seed)
    M = n_worlds
    counts = uneven_counts(rng, M, n_max)
    models = np.zeros(M, np.uint8)
    models[rng.permutation(M)[: M // 2]] = MODEL_ID
    fp = np.nonzero(models == MODEL_FP)[0]
    idw = np.nonzero(models == MODEL_ID)[0]
    P = empty_params(M)
    mass = MASS * rng.uniform(0.9, 1.1, size=len(fp))
    inertia = np.asarray(INERTIA)[None, :] * rng.uniform(0.9, 1.1, size=(len(fp), 3))
    fill_fp_airframe(P, fp, mass, inertia)
    gain, tau = _id_world_response(rng, len(idw))
    fill_id_model(P, idw, gain, tau)
    D = int(counts.sum())
    off = np.zeros(M + 1, np.int64)
    off[1:] = np.cumsum(counts)
    x0 = np.zeros((S_FP_PID, D))
    cmds = np.zeros((4, D))
    world_mass = P["mass"][:, 0]
    for w in range(M):
        n = int(counts[w])
        s = slice(off[w], off[w + 1])
        pos = _grid_positions(rng, n)
        if models[w] == MODEL_FP:
            x0[:, s] = _fp_pid_x0(n, np.full(n, world_mass[w]), pos)
            cmds[:, s] = _attitude_cmds(rng, n)
        else:
            x0[:S_ID, s] = _id_x0(n, pos)
            cmds[:, s] = _id_cmds(rng, n)
    return Workload("uneven_mixed", M, counts, models, CTRL_ATT_PID, INTEG_RK4,
                    float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(cmds))


def subset(w: Workload, worlds) -> Workload:
    """The workload restricted to the given worlds (in the given order)."""
    worlds = np.asarray(worlds)
    off = w.world_offsets()
    cols = np.concatenate([np.arange(off[i], off[i + 1]) for i in worlds]) if len(worlds) else np.zeros(0, np.int64)
    cmds = w.cmds[..., cols]
    return dataclasses.replace(
        w, n_worlds=len(worlds), drones_per_world=w.drones_per_world[worlds].copy(),
        model_per_world=w.model_per_world[worlds].copy(),
        params={k: v[worlds].copy() for k, v in w.params.items()},
        x0=np.ascontiguousarray(w.x0[:, cols]), cmds=np.ascontiguousarray(cmds),
        gain_index=None if w.gain_index is None else w.gain_index[worlds].copy(),
        ref_offset=None if w.ref_offset is None else np.ascontiguousarray(w.ref_offset[:, cols]),
        ref_time_shift=None if w.ref_time_shift is None else w.ref_time_shift[cols].copy(),
        dloss=None if w.dloss is None else w.dloss[cols].copy())


def uneven_mixed_adjoint(seed: int = 1005, n_worlds: int = 2048, n_subset: int = 256,
                    steps: int = 1000, dt: float = 0.002, n_max: int = 4000,
                    gain_std: float = 0.01) -> Workload:
    """The seeded world subset of the uneven batch that is differentiated: per-step
    commands (hover + noise), per-drone figure-eight offsets at the drones' start
    positions, one feedback gain per model (index 0 first-principles, 1 identified)."""
    base = uneven_mixed(seed, n_worlds, 1, dt, n_max)
    rng = _rng(seed + 7919)
    pick = np.sort(rng.permutation(n_worlds)[:n_subset])
    w = subset(base, pick)
    D = w.n_drones_total
    off = w.world_offsets()
    ubar = np.zeros((steps, 4, D))
    for i in range(w.n_worlds):
        s = slice(off[i], off[i + 1])
        if w.model_per_world[i] == MODEL_FP:
            ubar[:, 3, s] = float(w.params["mass"][i, 0]) * GRAVITY
        else:
            ubar[:, 3, s] = MASS * GRAVITY / ID_CF
    ubar += rng.normal(0.0, 0.02, size=ubar.shape)
    gain = rng.normal(0.0, gain_std, size=(2, 4, 13))
    gidx = np.where(w.model_per_world == MODEL_FP, 0, 1).astype(np.int32)
    return dataclasses.replace(
        w, name="uneven_mixed_adjoint", steps=steps, cmds=_f32(ubar), gain=_f32(gain),
        gain_index=gidx, ref_amp=1.0, ref_period=4.0, ref_offset=_f32(w.x0[0:3]),
        w_u=1e-3, dloss=np.ones(D, np.float32))


def mlp_policy_params(rng, n_policies: int, hidden: int, out_scale: float = 0.01) -> np.ndarray:
    """Random small-MLP policies [G, P], packed [W1 (H x 13) | b1 | W2 (H x H) | b2 |
    W3 (4 x H) | b3]: hidden weights N(0, 1/fan_in), output weights N(0, out_scale^2),
    biases 0 (a random draw and its layout only)."""
    H = int(hidden)
    out = []
    for _ in range(n_policies):
        out += [rng.normal(0.0, 1.0 / math.sqrt(13.0), size=13 * H), np.zeros(H),
                rng.normal(0.0, 1.0 / math.sqrt(H), size=H * H), np.zeros(H),
                rng.normal(0.0, out_scale, size=4 * H), np.zeros(4)]
    return _f32(np.concatenate(out).reshape(n_policies, -1))


def id_rollout_grad_mlp(seed: int = 1012, n_worlds: int = 1024, steps: int = 500, hidden: int = 32,
                dt: float = 0.002, out_scale: float = 0.01) -> Workload:
    """The differentiable workload with a small-MLP policy (width `hidden`) in place
    of the linear feedback gain."""
    w = id_rollout_grad(seed, n_worlds, steps, dt)
    rng = _rng(seed + 104729)
    return dataclasses.replace(w, name="id_rollout_grad_mlp", gain=mlp_policy_params(rng, 1, hidden, out_scale),
                               policy_hidden=int(hidden))


# command ranges of the normalised BPTT actions: +-0.5 rad on the attitude
# commands, +-0.9 of the hover thrust on the thrust command
BPTT_ACTION_RANGE = (0.5, 0.5, 0.5, 0.9 * MASS * GRAVITY / ID_CF)


def bptt_tracking(n_envs: int = 16, steps: int = 40, dt: float = 0.02, period: float = 10.0,
                  amp: float = 1.0, hidden: int = 0, seed: int = 1013, out_scale: float = 0.01) -> Workload:
    """The BPTT tracking setup shaped after the paper's (Methods, "Backpropagation
    Through Time"): ``n_envs`` identified-model drones with nominal parameters,
    start times spread evenly over one period of a figure-eight of period
    ``period`` (a 10 s closed trajectory), each drone starting exactly on the
    reference with its velocity and the hover thrust, no randomisation; per-step
    commands = the hover command, to which the policy adds its normalised action
    a = tanh(o) in [-1, 1] times BPTT_ACTION_RANGE; the paper's reward weights,
    which act on the normalised actions (so the raw-command weights are divided
    by the squared ranges). ``hidden`` = 0 gives a zero linear gain, > 0 a
    small-MLP policy drawn from ``seed``. Attitude commands at 1 / dt = 50 Hz."""
    M = D = n_envs
    P = empty_params(M)
    fill_id_model(P, np.arange(M), np.tile(ID_GAIN, (M, 1)), np.tile(ID_TAU, (M, 1)))
    shift = _f32(np.arange(D) * (period / D))
    s = shift.astype(np.float64)
    w0 = 2 * math.pi / period
    x0 = _id_x0(D, np.stack([amp * np.sin(w0 * s), 0.5 * amp * np.sin(2 * w0 * s), np.zeros(D)]))
    x0[6:9] = np.stack([amp * w0 * np.cos(w0 * s), amp * w0 * np.cos(2 * w0 * s), np.zeros(D)])
    ubar = np.zeros((steps, 4, D))
    ubar[:, 3] = MASS * GRAVITY / ID_CF
    if hidden:
        gain = mlp_policy_params(_rng(seed), 1, hidden, out_scale)
    else:
        gain = np.zeros((1, 4, 13))
    span = _f32(BPTT_ACTION_RANGE).astype(np.float64)
    reward = {"w_tilt": BPTT_REWARD["w_tilt"],
              "w_act": [float(np.float32(v / span[i] ** 2)) for i, v in enumerate(BPTT_REWARD["w_act"])],
              "w_dact": [float(np.float32(v / span[i] ** 2)) for i, v in enumerate(BPTT_REWARD["w_dact"])]}
    return Workload("id_bptt_tracking", M, np.ones(M, np.int32), np.full(M, MODEL_ID, np.uint8), CTRL_ATT_PID,
                    INTEG_RK4, float(np.float32(dt)), 1, _finish_params(P), _f32(x0), steps, _f32(ubar),
                    gain=_f32(gain), gain_index=None, ref_amp=amp, ref_period=period, ref_offset=None, w_u=0.0,
                    dloss=np.ones(D, np.float32), reward=reward, policy_hidden=int(hidden),
                    ref_time_shift=shift, policy_scale=_f32(BPTT_ACTION_RANGE))


def small(name: str, seed: int) -> Workload:
    """Reduced versions of the five workloads, by name, that the oracle finishes in
    seconds but that still span several 64-lane waves and a ragged tail."""
    if name == "fp_rotor_open_loop":
        return fp_rotor_open_loop(seed, n_worlds=16, steps=500)
    if name == "fp_pid_closed_loop":
        return fp_pid_closed_loop(seed, n_worlds=200, steps=1000)
    if name == "id_swarm":
        return id_swarm(seed, n_worlds=3, n_drones=150, steps=1000)
    if name == "id_rollout_grad":
        return id_rollout_grad(seed, n_worlds=100, steps=100)
    if name == "uneven_mixed":
        return uneven_mixed(seed, n_worlds=24, steps=300, n_max=120)
    raise ValueError(name)
