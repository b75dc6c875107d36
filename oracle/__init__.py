"""FP64 CPU oracle of the batched drone step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product path never does.
"""
from .dynamics import (  # noqa: F401
    MODEL_FP, MODEL_ID, CTRL_ROTOR, CTRL_ATT_PID, EULER, RK4,
    Batch, attitude_pid, body_z_in_world, euler_zyx_body_z, fp_rates, id_rates,
    integrate, per_drone_params, quat_mul, roll_pitch_from_quat, rollout, rollout_grad,
    rollout_workload, rotor_rates, rotor_speed_for_thrust, rotor_wrench, simulate_held,
    step_fp, step_id, t64,
)
