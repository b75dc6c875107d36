"""FP64 CPU oracle of the batched drone step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product path never does.
"""
from .dynamics import (  # noqa: F401
    MODEL_FP, MODEL_ID, CTRL_ROTOR, CTRL_ATT_PID, CTRL_TORQUE, CTRL_POSITION, EULER, RK4, allocate,
    position_controller,
    Batch, attitude_pid, body_z_in_world, drag_acceleration, euler_zyx_body_z, euler_zyx_matrix, fp_rates,
    id_rates, rotation_matrix,
    integrate, per_drone_params, quat_mul, roll_pitch_from_quat, rollout, rollout_grad,
    rollout_workload, rotor_rates, rotor_speed_for_thrust, rotor_wrench, simulate_held,
    step_fp, step_fp_multirate, step_id, t64, tilt_angle, hover_action, mlp_param_count, mlp_policy,
)
