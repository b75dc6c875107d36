// Layout constants shared by the host runtime and the kernels: the public
// per-world parameter record (fields of include/cfsim.h), the library-internal
// derived tail of the device copies, and the model / interface / integrator
// enums. Plain C++ (no HIP), so host-only code and its CPU tests can use it.
#pragma once

namespace cfk {

// parameter record offsets (public layout, see include/cfsim.h)
enum : int {
    P_MASS = 0, P_GRAVITY = 1, P_J = 2, P_THRUST = 5, P_TORQUE = 8, P_MIX_TX = 11,
    P_MIX_TY = 15, P_MIX_YAW = 19, P_MOTOR_UP = 23, P_MOTOR_DOWN = 25, P_JP = 27,
    P_DRAG = 28, P_ANG_KP = 31, P_ANG_KI = 33, P_RATE_KP = 35, P_RATE_KI = 38,
    P_RATE_KD = 41, P_J_CTRL = 44, P_F_MAX = 47, P_ALLOC = 48, P_CF = 64, P_CTAU = 65,
    P_CPSI1 = 66, P_CPSI2 = 69, P_CPSI3 = 72, P_POS_KP = 75, P_POS_KV = 78, P_ATT_KR = 81,
    P_ATT_KW = 84, NPARAM = 96
};
// Per-world constants derived on the host from the public record (library-internal
// tail of the device copies, which have NREC floats per world): reciprocals and
// the reference-speed terms of the first-principles model, the identified model's
// c_f / m and hover thrust. Kernels read them like the public fields instead of
// spending registers and instructions forming them.
enum : int {
    D_INV_M = 96, D_IJ = 97, D_DJ = 100, D_INV_2K2 = 103, D_SG = 104, D_WR = 108, D_W2 = 109,
    D_K1W = 110, D_T1W = 111, D_FR = 112, D_F4R = 113, D_TXR = 114, D_TYR = 115, D_TZR = 116,
    D_SGR = 117, D_DISC_R = 118, D_VTX = 119, D_CF_M = 120, D_F_HOVER = 121, D_TPROP = 122, D_TZK = 123,
    NREC = 128
};
enum : int { MODEL_FP = 0, MODEL_ID = 1 };
enum : int { CTRL_ROTOR = 0, CTRL_PID = 1, CTRL_TORQUE = 2, CTRL_POSITION = 3 };
enum : int { EULER = 0, RK4 = 1 };
constexpr int S_FP = 17, S_PID = 25, S_ID = 13;

}  // namespace cfk
