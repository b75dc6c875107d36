"""Batched drone simulation step for AMD MI355X (gfx950): HIP kernels behind a C
interface (include/cfsim.h) and a thin Python binding."""
from .binding import (  # noqa: F401
    CfError, Mppi, RolloutLoss, Sim, load, pack_params,
    MODEL_FP, MODEL_ID, CTRL_ROTOR, CTRL_ATT_PID, CTRL_TORQUE, CTRL_POSITION, INTEG_EULER, INTEG_RK4,
    F_PLAIN_KERNEL, F_NONFINITE_CHECK, F_GRAPH, F_WORKQUEUE, F_NO_AUTOTUNE_CACHE, F_SINGLE_LAUNCH,
)
from .bptt import train_linear_policy  # noqa: F401
