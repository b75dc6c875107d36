// Device-side model of the batched drone step for gfx950 (one drone per lane,
// everything in registers). Forward maps and their hand-written vector-Jacobian
// products (VJPs) for the discrete adjoint.
//
// Models (Crazyflow, arXiv 2606.01478, Methods):
//   first-principles: Eq. (1) rigid body + second-order thrust/drag-torque
//     polynomials + mixing matrix + adapted rotor dynamics (Eq. rotor_adapted);
//   identified: Eqs. 3_simplified_acceleration / _force / _rpy.
// Integration: explicit Euler or classical RK4, command held over the step,
// quaternion renormalised after the step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cf_layout.hpp"

namespace cfk {

// hardware square root, reciprocal square root and reciprocal (within 1 ulp on gfx950)
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsqrt_hw(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }


// Accessors over one world's record in the array-of-structs copy (uniform world
// per workgroup). Where the values live is a register-budget choice made per
// kernel by measurement: plain loads (the compiler decides); loads through the
// constant address space, which with a uniform pointer become scalar loads into
// scalar registers (the records are never written while kernels run) and free
// vector registers for the reverse step; forced per-lane vector loads for the
// sampled-rollout kernel, whose scalar registers hold its large argument block.
struct AosRec {
    const float* r;
    __device__ __forceinline__ float operator()(int i) const { return r[i]; }
};
typedef const __attribute__((address_space(4))) float const_float;
struct ScalarRec {
    const float* r;
    __device__ __forceinline__ float operator()(int i) const { return ((const_float*)r)[i]; }
};
// every field through per-lane vector loads even where the pointer is uniform
// (an offset the compiler cannot see to be zero), for kernels whose scalar
// registers are already full with kernel arguments
struct VecRec {
    const float* r;
    int zero;
    __device__ __forceinline__ explicit VecRec(const float* rec) : r(rec) {
        asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    }
    __device__ __forceinline__ float operator()(int i) const { return r[i + zero]; }
};
// accessor over a world's record in the transposed [NREC][M] copy (per-lane world)
struct SoaRec {
    const float* p; int M; int w;
    __device__ __forceinline__ float operator()(int i) const { return p[(size_t)i * M + w]; }
};

// The record with its base pointer hidden from the optimiser: loads through the
// copy are issued where they are written (e.g. once per controller evaluation)
// instead of being hoisted out of the step loop and held in registers across it.
// A uniform record's copy reads through the constant address space (scalar
// loads), since the pointer the optimiser cannot follow would otherwise take
// generic vector loads.
__device__ __forceinline__ ScalarRec laundered(AosRec r) {
    asm volatile("" : "+s"(r.r));
    return ScalarRec{r.r};
}
__device__ __forceinline__ SoaRec laundered(SoaRec r) {
    asm volatile("" : "+s"(r.p));
    return r;
}
__device__ __forceinline__ ScalarRec laundered(ScalarRec r) {
    asm volatile("" : "+s"(r.r));
    return r;
}

// a world record whose address differs across the lanes of a wave (a packed
// tile across a world boundary): per-lane vector loads
struct LaneRec {
    const float* r;
    __device__ __forceinline__ float operator()(int i) const {
        return ((const __attribute__((address_space(1))) float*)r)[i];
    }
};
__device__ __forceinline__ LaneRec laundered(LaneRec r) {
    asm volatile("" : "+v"(r.r));
    return r;
}

struct FpParams {
    float inv_m, g;
    float iJx, iJy, iJz, dJx, dJy, dJz;  // dJx = Jz - Jy, dJy = Jx - Jz, dJz = Jy - Jx
    float k2, t2, inv_2k2;
    float tx[4], ty[4], tz[4];
    float cvu, cdu, cvd, cdd;
    float jp, sg[4];          // propeller inertia, rotor spin directions (-sign of the yaw mixing)
    float cd[3];              // linear drag C_a diagonal
    bool gyro, drag;          // J_p != 0, C_a != 0
    // rotor law with distinct acceleration / deceleration coefficients or a
    // quadratic term; otherwise W' = c_v (W_cmd - W) on both branches
    bool rotor_general;
    // drag torque = kappa * thrust for every rotor: the yaw torque is formed from
    // the thrust differences with coefficients tzk = kappa * yaw mixing
    bool tprop;
    float tzk[4];
    // Inside the kernels the four rotor rows hold W - W_r, the deviation from a
    // reference speed W_r (the world's hover speed), and rotor commands are
    // deviations too: near 15 000 an FP32 speed resolves 1e-3, its deviation
    // resolves 1e-4 or better, and the body torques are differences of rotor
    // thrusts. Thrust and drag torque are evaluated as differences from their
    // values at W_r.
    float wr;                 // W_r
    float w2;                 // 2 W_r
    float k1w, t1w;           // k1 + 2 k2 W_r, t1 + 2 t2 W_r
    float fr;                 // thrust of one rotor at W_r
    float F4r, txr, tyr, tzr; // 4 fr, fr sum tx, fr sum ty, tr sum tz
    float sgr;                // W_r sum sigma
    float disc_r;             // discriminant of the thrust curve at fr: (k1 + 2 k2 W_r)^2
    float vtx;                // the curve's vertex as a deviation: -(k1 + 2 k2 W_r) / (2 k2)
};
struct PidParams {
    float akp[2], aki[2], rkp[3], rki[3], rkd[3], jc[3], fmax;
    float A[16];
    // position interface (geometric controller): mass, gravity and gains
    float m, g, pkp[3], pkv[3], akr[3], akw[3];
};
struct IdParams {
    float cf_m, g, ctau, f_hover, inv_m;
    float c1[3], c2[3], c3[3];
    float cd[3];
    bool drag;
    bool direct;  // c_tau = 0: no thrust dynamics, the commanded thrust acts directly
};

// AERO = false: the gyroscopic/reaction torques, drag and the general rotor law
// (distinct acceleration / deceleration coefficients, quadratic term) are
// compiled out (the flags below become constants and their branches fold away)
template <bool AERO, class R>
__device__ __forceinline__ FpParams load_fp(const R& rec) {
    FpParams P;
    P.inv_m = rec(D_INV_M);
    P.g = rec(P_GRAVITY);
    P.iJx = rec(D_IJ); P.iJy = rec(D_IJ + 1); P.iJz = rec(D_IJ + 2);
    P.dJx = rec(D_DJ); P.dJy = rec(D_DJ + 1); P.dJz = rec(D_DJ + 2);
    P.k2 = rec(P_THRUST + 2);
    P.t2 = rec(P_TORQUE + 2);
    P.inv_2k2 = rec(D_INV_2K2);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        P.tx[i] = rec(P_MIX_TX + i); P.ty[i] = rec(P_MIX_TY + i); P.tz[i] = rec(P_MIX_YAW + i);
    }
    P.cvu = rec(P_MOTOR_UP);
    if constexpr (AERO) {
        P.cdu = rec(P_MOTOR_UP + 1);
        P.cvd = rec(P_MOTOR_DOWN); P.cdd = rec(P_MOTOR_DOWN + 1);
        P.rotor_general = (P.cdu != 0.f) || (P.cdd != 0.f) || (P.cvd != P.cvu);
        P.tprop = rec(D_TPROP) != 0.f;
        P.jp = rec(P_JP);
#pragma unroll
        for (int i = 0; i < 4; ++i) P.sg[i] = rec(D_SG + i);
#pragma unroll
        for (int i = 0; i < 3; ++i) P.cd[i] = rec(P_DRAG + i);
        P.gyro = P.jp != 0.f;
        P.drag = (P.cd[0] != 0.f) || (P.cd[1] != 0.f) || (P.cd[2] != 0.f);
        P.sgr = rec(D_SGR);
    } else {
        P.jp = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) P.sg[i] = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) P.cd[i] = 0.f;
        P.gyro = false;
        P.drag = false;
        P.sgr = 0.f;
        P.cdu = 0.f; P.cvd = P.cvu; P.cdd = 0.f;
        P.rotor_general = false;
        P.tprop = true;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) P.tzk[i] = rec(D_TZK + i);
    P.wr = rec(D_WR);
    P.w2 = rec(D_W2);
    P.k1w = rec(D_K1W);
    P.t1w = rec(D_T1W);
    P.fr = rec(D_FR);
    P.F4r = rec(D_F4R);
    P.txr = rec(D_TXR);
    P.tyr = rec(D_TYR);
    P.tzr = rec(D_TZR);
    P.disc_r = rec(D_DISC_R);
    P.vtx = rec(D_VTX);
    return P;
}

// rotor rows 13..16 between the absolute speeds of the public state layout and
// the in-register deviations
__device__ __forceinline__ void rotors_to_dev(float* x, const FpParams& P) {
#pragma unroll
    for (int i = 0; i < 4; ++i) x[13 + i] -= P.wr;
}
__device__ __forceinline__ void rotors_from_dev(float* x, const FpParams& P) {
#pragma unroll
    for (int i = 0; i < 4; ++i) x[13 + i] += P.wr;
}

template <class R>
__device__ __forceinline__ PidParams load_pid(const R& rec, bool position) {
    PidParams C;
    if (position) {
        C.m = rec(P_MASS);
        C.g = rec(P_GRAVITY);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            C.pkp[i] = rec(P_POS_KP + i); C.pkv[i] = rec(P_POS_KV + i);
            C.akr[i] = rec(P_ATT_KR + i); C.akw[i] = rec(P_ATT_KW + i);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) { C.akp[i] = rec(P_ANG_KP + i); C.aki[i] = rec(P_ANG_KI + i); }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        C.rkp[i] = rec(P_RATE_KP + i); C.rki[i] = rec(P_RATE_KI + i);
        C.rkd[i] = rec(P_RATE_KD + i); C.jc[i] = rec(P_J_CTRL + i);
    }
    C.fmax = rec(P_F_MAX);
#pragma unroll
    for (int i = 0; i < 16; ++i) C.A[i] = rec(P_ALLOC + i);
    return C;
}

template <bool AERO, class R>
__device__ __forceinline__ IdParams load_id(const R& rec) {
    IdParams P;
    P.cf_m = rec(D_CF_M);
    P.g = rec(P_GRAVITY);
    P.ctau = rec(P_CTAU);
    P.direct = P.ctau == 0.f;
    P.f_hover = rec(D_F_HOVER);
    P.inv_m = rec(D_INV_M);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        P.c1[i] = rec(P_CPSI1 + i); P.c2[i] = rec(P_CPSI2 + i); P.c3[i] = rec(P_CPSI3 + i);
        P.cd[i] = AERO ? rec(P_DRAG + i) : 0.f;
    }
    P.drag = AERO && ((P.cd[0] != 0.f) || (P.cd[1] != 0.f) || (P.cd[2] != 0.f));
    return P;
}

// ---------------------------------------------------------------------------
// elementary functions

// sin and cos of x together: Cody and Waite's argument reduction by pi/2 with a
// three-part constant (r = x - k pi/2, |r| <= pi/4), Taylor polynomials of
// degree 9 (sin) and 10 (cos) in r (truncation below 2e-9), and the quadrant
// of k. About 1.4 ulp for |x| <= 2^15.
__device__ __forceinline__ void sincos_cw(float x, float* s, float* c) {
    const float k = __builtin_rintf(x * 0x1.45f306p-1f);          // x * 2/pi
    float r = __builtin_fmaf(-k, 0x1.921fb6p+0f, x);              // pi/2, leading part
    r = __builtin_fmaf(-k, -0x1.777a5cp-25f, r);                  // second part
    r = __builtin_fmaf(-k, -0x1.0p-49f, r);                       // third part
    const float z = r * r;
    float ps = __builtin_fmaf(z, 0x1.71de3ap-19f, -0x1.a01a02p-13f);  // 1/9!, -1/7!
    ps = __builtin_fmaf(z, ps, 0x1.111112p-7f);                        // 1/5!
    ps = __builtin_fmaf(z, ps, -0x1.555556p-3f);                       // -1/3!
    const float sv = __builtin_fmaf(r * z, ps, r);
    float pc = __builtin_fmaf(z, -0x1.27e4fcp-22f, 0x1.a01a02p-16f);  // -1/10!, 1/8!
    pc = __builtin_fmaf(z, pc, -0x1.6c16c2p-10f);                      // -1/6!
    pc = __builtin_fmaf(z, pc, 0x1.555556p-5f);                        // 1/4!
    pc = __builtin_fmaf(z, pc, -0.5f);
    const float cv = __builtin_fmaf(z, pc, 1.0f);
    const int q = (int)k;
    float sr = (q & 1) ? cv : sv;
    float cr = (q & 1) ? sv : cv;
    *s = (q & 2) ? -sr : sr;
    *c = ((q + 1) & 2) ? -cr : cr;
}

// atan2(y, x): octant reduction to t = min(|x|, |y|) / max(|x|, |y|) in [0, 1],
// atan(t) = t p(t^2) with p of degree 8, then the octant's reflections
// (pi/2 - a, pi - a, sign of y). The coefficients are a relative-error minimax
// fit of atan(sqrt(s)) / sqrt(s) on s in [0, 1] made for this library (Lawson's
// iteratively reweighted least squares, rounded to binary32): at most 1.9 ulp
// and 1.2e-7 rad on [0, 1] with this Horner evaluation. atan2(0, 0) = 0.
__device__ __forceinline__ float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.f ? mn * rcp_hw(mx) : 0.f;
    const float s = t * t;
    float p = 0x1.7c938cp-9f;                      //  2.9035672e-3
    p = __builtin_fmaf(p, s, -0x1.0ac82ap-6f);     // -1.6283074e-2
    p = __builtin_fmaf(p, s, 0x1.60945ap-5f);      //  4.3039490e-2
    p = __builtin_fmaf(p, s, -0x1.349472p-4f);     // -7.5336881e-2
    p = __builtin_fmaf(p, s, 0x1.b46a76p-4f);      //  1.0654684e-1
    p = __builtin_fmaf(p, s, -0x1.22f64ep-3f);     // -1.4207135e-1
    p = __builtin_fmaf(p, s, 0x1.99753p-3f);       //  1.9993055e-1
    p = __builtin_fmaf(p, s, -0x1.5554b4p-2f);     // -3.3333093e-1
    p = __builtin_fmaf(p, s, 1.0f);
    float a = t * p;
    if (ay > ax) a = 0x1.921fb6p+0f - a;           // pi/2
    if (x < 0.f) a = 0x1.921fb6p+1f - a;           // pi
    return copysignf(a, y);
}

// asin(x) for |x| <= 1 as atan2(x, sqrt((1 - x)(1 + x)))
__device__ __forceinline__ float asin_poly(float x) {
    return atan2_poly(x, sqrt_hw((1.f - x) * (1.f + x)));
}

// sines and cosines of the three Euler angles; arguments beyond 2^15 rad (never
// reached by the workloads) take the library routine for all three
__device__ __forceinline__ void sincos3(const float* a, float* s, float* c) {
    const float m = fmaxf(fabsf(a[0]), fmaxf(fabsf(a[1]), fabsf(a[2])));
    if (__builtin_expect(m > 32768.f, 0)) {
#pragma unroll
        for (int i = 0; i < 3; ++i) sincosf(a[i], s + i, c + i);
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) sincos_cw(a[i], s + i, c + i);
    }
}

// Euler-angle trigonometry of RK4 stage states. A stage's angles differ from
// the step's start angles a0 by a small offset d (h/2 or h times a stage
// rate), so sin and cos follow from those at a0 by the angle-addition
// formulas with short series for sin d and cos d - 1 (|d| <= 1/16: the
// truncation is below 1e-12); a larger offset anywhere in the wave takes
// sincos3. Stage 1 (d = 0) returns the start values exactly.
struct EulerBase {
    float a0[3], s0[3], c0[3];
};

__device__ __forceinline__ void euler_base(const float* a, EulerBase& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i) b.a0[i] = a[i];
    sincos3(a, b.s0, b.c0);
}

__device__ __forceinline__ void sincos3_near(const float* a, const EulerBase& b, float* s, float* c) {
    float d[3];
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] = a[i] - b.a0[i];
        m = fmaxf(m, fabsf(d[i]));
    }
    if (m <= 0.0625f) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float d2 = d[i] * d[i];
            const float sd = __builtin_fmaf(d[i] * d2, __builtin_fmaf(d2, 1.f / 120.f, -1.f / 6.f), d[i]);
            const float cm1 = d2 * __builtin_fmaf(d2, __builtin_fmaf(d2, -1.f / 720.f, 1.f / 24.f), -0.5f);
            s[i] = __builtin_fmaf(b.s0[i], cm1, __builtin_fmaf(b.c0[i], sd, b.s0[i]));
            c[i] = __builtin_fmaf(b.c0[i], cm1, __builtin_fmaf(-b.s0[i], sd, b.c0[i]));
        }
    } else {
        sincos3(a, s, c);
    }
}

// ---------------------------------------------------------------------------
// rotation matrices (row-major 3x3) and the linear drag term R C_a R^T v / m

// body->world matrix of a unit quaternion (x, y, z, w), used on stage
// quaternions as they are
__device__ __forceinline__ void quat_matrix(float x, float y, float z, float w, float* R) {
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

// qb += (dR/dq)^T Rb
__device__ __forceinline__ void quat_matrix_vjp(float x, float y, float z, float w, const float* Rb, float* qb) {
    qb[0] += 2.f * (y * Rb[1] + z * Rb[2] + y * Rb[3] - w * Rb[5] + z * Rb[6] + w * Rb[7]) - 4.f * x * (Rb[4] + Rb[8]);
    qb[1] += 2.f * (x * Rb[1] + w * Rb[2] + x * Rb[3] + z * Rb[5] - w * Rb[6] + z * Rb[7]) - 4.f * y * (Rb[0] + Rb[8]);
    qb[2] += 2.f * (-w * Rb[1] + x * Rb[2] + w * Rb[3] + y * Rb[5] + x * Rb[6] + y * Rb[7]) - 4.f * z * (Rb[0] + Rb[4]);
    qb[3] += 2.f * (-z * Rb[1] + y * Rb[2] + z * Rb[3] - x * Rb[5] - y * Rb[6] + x * Rb[7]);
}

// R = Rz(yaw) Ry(pitch) Rx(roll) from the sines/cosines of (roll, pitch, yaw)
__device__ __forceinline__ void euler_matrix(const float* sn, const float* cs, float* R) {
    const float sf = sn[0], cf = cs[0], st = sn[1], ct = cs[1], sp = sn[2], cp = cs[2];
    R[0] = cp * ct; R[1] = cp * st * sf - sp * cf; R[2] = cp * st * cf + sp * sf;
    R[3] = sp * ct; R[4] = sp * st * sf + cp * cf; R[5] = sp * st * cf - cp * sf;
    R[6] = -st;     R[7] = ct * sf;                R[8] = ct * cf;
}

// psib += (dR/dPsi)^T Rb
__device__ __forceinline__ void euler_matrix_vjp(const float* sn, const float* cs, const float* Rb, float* psib) {
    const float sf = sn[0], cf = cs[0], st = sn[1], ct = cs[1], sp = sn[2], cp = cs[2];
    psib[0] += Rb[1] * (cp * st * cf + sp * sf) + Rb[2] * (-cp * st * sf + sp * cf) +
               Rb[4] * (sp * st * cf - cp * sf) + Rb[5] * (-sp * st * sf - cp * cf) + Rb[7] * (ct * cf) -
               Rb[8] * (ct * sf);
    psib[1] += -Rb[0] * (cp * st) + Rb[1] * (cp * ct * sf) + Rb[2] * (cp * ct * cf) - Rb[3] * (sp * st) +
               Rb[4] * (sp * ct * sf) + Rb[5] * (sp * ct * cf) - Rb[6] * ct - Rb[7] * (st * sf) - Rb[8] * (st * cf);
    psib[2] += -Rb[0] * (sp * ct) + Rb[1] * (-sp * st * sf - cp * cf) + Rb[2] * (-sp * st * cf + cp * sf) +
               Rb[3] * (cp * ct) + Rb[4] * (cp * st * sf - sp * cf) + Rb[5] * (cp * st * cf + sp * sf);
}

// acc += R diag(cd) R^T v / m
__device__ __forceinline__ void drag_acc(const float* R, const float* v, const float* cd, float inv_m, float* acc) {
    float fb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) fb[j] = cd[j] * (R[j] * v[0] + R[3 + j] * v[1] + R[6 + j] * v[2]) * inv_m;
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] += R[3 * i] * fb[0] + R[3 * i + 1] * fb[1] + R[3 * i + 2] * fb[2];
}

// VJP of drag_acc w.r.t. v (vb +=) and R (Rb +=), given the adjoint ga of acc
__device__ __forceinline__ void drag_acc_vjp(const float* R, const float* v, const float* cd, float inv_m,
                                             const float* ga, float* vb, float* Rb) {
    float vbody[3], fb[3], fbb[3], vbb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        vbody[j] = R[j] * v[0] + R[3 + j] * v[1] + R[6 + j] * v[2];
        fb[j] = cd[j] * vbody[j] * inv_m;
        fbb[j] = R[j] * ga[0] + R[3 + j] * ga[1] + R[6 + j] * ga[2];   // R^T ga
        vbb[j] = cd[j] * inv_m * fbb[j];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        vb[i] += R[3 * i] * vbb[0] + R[3 * i + 1] * vbb[1] + R[3 * i + 2] * vbb[2];
#pragma unroll
        for (int j = 0; j < 3; ++j) Rb[3 * i + j] += ga[i] * fb[j] + v[i] * vbb[j];
    }
}

// ---------------------------------------------------------------------------
// first-principles right-hand side, 17 components [p q v w Omega]
__device__ __forceinline__ void fp_rates(const float* x, const float* rc, const FpParams& P, float* xd) {
    const float qx = x[3], qy = x[4], qz = x[5], qw = x[6];
    const float wx = x[10], wy = x[11], wz = x[12];
    // rotor rows and commands are deviations from W_r (see FpParams); the sums
    // start from the wrench of four rotors at W_r
    float F = P.F4r, tx = P.txr, ty = P.tyr, tz = P.tzr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = x[13 + i];
        const float e = rc[i] - r;            // W_cmd - W
        if (P.rotor_general) {
            const bool up = e >= 0.f;         // accelerating branch (ties included)
            const float cv = up ? P.cvu : P.cvd;
            const float cd = up ? P.cdu : P.cdd;
            xd[13 + i] = e * (cv + cd * (P.w2 + rc[i] + r));   // c_v e + c_d (W_cmd^2 - W^2)
        } else {
            xd[13 + i] = P.cvu * e;
        }
        const float df = r * (P.k1w + P.k2 * r);           // f(W) - f(W_r)
        F += df;
        tx += P.tx[i] * df;
        ty += P.ty[i] * df;
        if (P.tprop) {
            tz += P.tzk[i] * df;
        } else {
            const float dq = r * (P.t1w + P.t2 * r);
            tz += P.tz[i] * dq;
        }
    }
    xd[0] = x[7]; xd[1] = x[8]; xd[2] = x[9];
    xd[3] = 0.5f * (qw * wx + qy * wz - qz * wy);
    xd[4] = 0.5f * (qw * wy + qz * wx - qx * wz);
    xd[5] = 0.5f * (qw * wz + qx * wy - qy * wx);
    xd[6] = -0.5f * (qx * wx + qy * wy + qz * wz);
    const float a = F * P.inv_m;
    xd[7] = a * (2.f * (qx * qz + qw * qy));
    xd[8] = a * (2.f * (qy * qz - qw * qx));
    xd[9] = a * (1.f - 2.f * (qx * qx + qy * qy)) - P.g;
    if (P.drag) {
        float R[9];
        quat_matrix(qx, qy, qz, qw, R);
        drag_acc(R, x + 7, P.cd, P.inv_m, xd + 7);
    }
    if (P.gyro) {
        // -w x h - h', h = J_p Omega_s e_z, Omega_s = sum sigma_i Omega_i
        float om_s = P.sgr, dom_s = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            om_s += P.sg[i] * x[13 + i];
            dom_s += P.sg[i] * xd[13 + i];
        }
        tx -= P.jp * wy * om_s;
        ty += P.jp * wx * om_s;
        tz -= P.jp * dom_s;
    }
    xd[10] = (tx - P.dJx * wy * wz) * P.iJx;
    xd[11] = (ty - P.dJy * wz * wx) * P.iJy;
    xd[12] = (tz - P.dJz * wx * wy) * P.iJz;
}

// VJP of fp_rates at (x, rc): xb += (d xd/d x)^T gb, rcb += (d xd/d rc)^T gb
__device__ __forceinline__ void fp_rates_vjp(const float* x, const float* rc, const FpParams& P,
                                             const float* gb, float* xb, float* rcb) {
    const float qx = x[3], qy = x[4], qz = x[5], qw = x[6];
    const float wx = x[10], wy = x[11], wz = x[12];
    float F = P.F4r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = x[13 + i];
        F += r * (P.k1w + P.k2 * r);
    }
    // p' = v
    xb[7] += gb[0]; xb[8] += gb[1]; xb[9] += gb[2];
    // q' = 1/2 q (x) [w, 0]
    const float gx = gb[3], gy = gb[4], gz = gb[5], gw = gb[6];
    xb[3] += 0.5f * (-gy * wz + gz * wy - gw * wx);
    xb[4] += 0.5f * (gx * wz - gz * wx - gw * wy);
    xb[5] += 0.5f * (-gx * wy + gy * wx - gw * wz);
    xb[6] += 0.5f * (gx * wx + gy * wy + gz * wz);
    xb[10] += 0.5f * (qw * gx + qz * gy - qy * gz - qx * gw);
    xb[11] += 0.5f * (-qz * gx + qw * gy + qx * gz - qy * gw);
    xb[12] += 0.5f * (qy * gx - qx * gy + qw * gz - qz * gw);
    // v' = (F/m) R(q) e_z - g e_z
    const float rz0 = 2.f * (qx * qz + qw * qy);
    const float rz1 = 2.f * (qy * qz - qw * qx);
    const float rz2 = 1.f - 2.f * (qx * qx + qy * qy);
    const float a = F * P.inv_m;
    const float Fb = (gb[7] * rz0 + gb[8] * rz1 + gb[9] * rz2) * P.inv_m;
    const float r0b = a * gb[7], r1b = a * gb[8], r2b = a * gb[9];
    xb[3] += 2.f * (qz * r0b - qw * r1b) - 4.f * qx * r2b;
    xb[4] += 2.f * (qw * r0b + qz * r1b) - 4.f * qy * r2b;
    xb[5] += 2.f * (qx * r0b + qy * r1b);
    xb[6] += 2.f * (qy * r0b - qx * r1b);
    if (P.drag) {
        float R[9], Rb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        quat_matrix(qx, qy, qz, qw, R);
        drag_acc_vjp(R, x + 7, P.cd, P.inv_m, gb + 7, xb + 7, Rb);
        quat_matrix_vjp(qx, qy, qz, qw, Rb, xb + 3);
    }
    // w' = (tau - w x J w) / J
    const float hx = gb[10] * P.iJx, hy = gb[11] * P.iJy, hz = gb[12] * P.iJz;
    xb[10] -= hy * P.dJy * wz + hz * P.dJz * wy;
    xb[11] -= hx * P.dJx * wz + hz * P.dJz * wx;
    xb[12] -= hx * P.dJx * wy + hy * P.dJy * wx;
    float om_sb = 0.f;
    if (P.gyro) {
        float om_s = P.sgr;
#pragma unroll
        for (int i = 0; i < 4; ++i) om_s += P.sg[i] * x[13 + i];
        xb[11] -= P.jp * om_s * hx;
        xb[10] += P.jp * om_s * hy;
        om_sb = P.jp * (wx * hy - wy * hx);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = x[13 + i];
        const float fb = Fb + P.tx[i] * hx + P.ty[i] * hy + (P.tprop ? P.tzk[i] * hz : 0.f);
        const float tqb = P.tprop ? 0.f : P.tz[i] * hz;
        // adjoint of the rotor acceleration: the state derivative, plus the reaction torque
        const float gr = gb[13 + i] - (P.gyro ? P.jp * P.sg[i] * hz : 0.f);
        if (P.gyro) xb[13 + i] += P.sg[i] * om_sb;
        // df/dW = k1 + 2 k2 W = k1w + 2 k2 r, d(W^2)/dW = 2 W = w2 + 2 r
        xb[13 + i] += fb * (P.k1w + 2.f * P.k2 * r);
        if (!P.tprop) xb[13 + i] += tqb * (P.t1w + 2.f * P.t2 * r);
        if (P.rotor_general) {
            const bool up = rc[i] - r >= 0.f;
            const float cv = up ? P.cvu : P.cvd;
            const float cd = up ? P.cdu : P.cdd;
            xb[13 + i] -= gr * (cv + cd * (P.w2 + 2.f * r));
            rcb[i] += gr * (cv + cd * (P.w2 + 2.f * rc[i]));
        } else {
            xb[13 + i] -= gr * P.cvu;
            rcb[i] += gr * P.cvu;
        }
    }
}

// ---------------------------------------------------------------------------
// identified model right-hand side, 13 components [p Psi v dPsi f]
// AT_BASE: x holds the base angles themselves (an RK4 step's first stage), whose
// sines and cosines B already holds (the angle-addition form returns exactly
// these at a zero offset)
template <bool AT_BASE = false>
__device__ __forceinline__ void id_rates(const float* x, const float* u, const IdParams& P, const EulerBase& B,
                                         float* xd) {
    float sn[3], cs[3];
    if constexpr (AT_BASE) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { sn[i] = B.s0[i]; cs[i] = B.c0[i]; }
    } else {
        sincos3_near(x + 3, B, sn, cs);
    }
    const float sph = sn[0], cph = cs[0], sth = sn[1], cth = cs[1], sps = sn[2], cps = cs[2];
    const float a = P.cf_m * (P.direct ? u[3] : x[12]);
    xd[0] = x[6]; xd[1] = x[7]; xd[2] = x[8];
    xd[3] = x[9]; xd[4] = x[10]; xd[5] = x[11];
    xd[6] = a * (cps * sth * cph + sps * sph);
    xd[7] = a * (sps * sth * cph - cps * sph);
    xd[8] = a * (cth * cph) - P.g;
    if (P.drag) {
        float R[9];
        euler_matrix(sn, cs, R);
        drag_acc(R, x + 6, P.cd, P.inv_m, xd + 6);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) xd[9 + i] = P.c1[i] * x[3 + i] + P.c2[i] * x[9 + i] + P.c3[i] * u[i];
    xd[12] = P.ctau * (u[3] - x[12]);
}

template <bool AT_BASE = false>
__device__ __forceinline__ void id_rates_vjp(const float* x, const float* u, const IdParams& P, const EulerBase& B,
                                             const float* gb, float* xb, float* ub) {
    float sn[3], cs[3];
    if constexpr (AT_BASE) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { sn[i] = B.s0[i]; cs[i] = B.c0[i]; }
    } else {
        sincos3_near(x + 3, B, sn, cs);
    }
    const float sph = sn[0], cph = cs[0], sth = sn[1], cth = cs[1], sps = sn[2], cps = cs[2];
    const float a = P.cf_m * (P.direct ? u[3] : x[12]);
    const float rz0 = cps * sth * cph + sps * sph;
    const float rz1 = sps * sth * cph - cps * sph;
    const float rz2 = cth * cph;
    // p' = v, Psi' = dPsi
    xb[6] += gb[0]; xb[7] += gb[1]; xb[8] += gb[2];
    xb[9] += gb[3]; xb[10] += gb[4]; xb[11] += gb[5];
    // v' = a R e_z - g e_z, a = c_f f / m with f the thrust state or (direct) the command
    const float fb = (gb[6] * rz0 + gb[7] * rz1 + gb[8] * rz2) * P.cf_m;
    if (P.direct) ub[3] += fb;
    else xb[12] += fb;
    const float b0 = a * gb[6], b1 = a * gb[7], b2 = a * gb[8];
    xb[3] += b0 * (sps * cph - cps * sth * sph) + b1 * (-sps * sth * sph - cps * cph) + b2 * (-cth * sph);
    xb[4] += b0 * (cps * cth * cph) + b1 * (sps * cth * cph) + b2 * (-sth * cph);
    xb[5] += b0 * (cps * sph - sps * sth * cph) + b1 * (cps * sth * cph + sps * sph);
    if (P.drag) {
        float R[9], Rb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        euler_matrix(sn, cs, R);
        drag_acc_vjp(R, x + 6, P.cd, P.inv_m, gb + 6, xb + 6, Rb);
        euler_matrix_vjp(sn, cs, Rb, xb + 3);
    }
    // Psi'' = c1 Psi + c2 dPsi + c3 Psi_cmd
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float h = gb[9 + i];
        xb[3 + i] += P.c1[i] * h;
        xb[9 + i] += P.c2[i] * h;
        ub[i] += P.c3[i] * h;
    }
    // f' = c_tau (f_cmd - f)
    xb[12] -= P.ctau * gb[12];
    ub[3] += P.ctau * gb[12];
}

// ---------------------------------------------------------------------------
// cascaded attitude PID + allocation (project design; evaluated once per step)
struct PidTrace {
    float s1, c1, s2, disc[4];
    bool pass[4];   // allocated thrust inside [0, f_max] on the rising branch
};

// Motor allocation: f = alloc [T, tau_x, tau_y, tau_z], clamped to [0, f_max],
// rotor-speed commands from the thrust curve. Also the torque interface.
// Commands are deviations xi from W_r: f(W_r + xi) = f is
// xi (k1 + 2 k2 W_r + k2 xi) = f - f_r, solved as
// xi = 2 (f - f_r) / (sqrt(disc) + k1 + 2 k2 W_r), disc = (k1 + 2 k2 W_r)^2 + 4 k2 (f - f_r),
// which has no cancellation; f - f_r is formed with the thrust term fused.
__device__ __forceinline__ void allocate(const float* wrench, const FpParams& P, const PidParams& C, float* rc,
                                         PidTrace& tr) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float dfr = fmaf(C.A[4 * j], wrench[0], -P.fr) +
                          (C.A[4 * j + 1] * wrench[1] + C.A[4 * j + 2] * wrench[2] + C.A[4 * j + 3] * wrench[3]);
        const float lo = -P.fr, hi = C.fmax - P.fr;
        const float df = fminf(fmaxf(dfr, lo), hi);
        const float disc = fmaf(4.f * P.k2, df, P.disc_r);
        tr.disc[j] = disc;
        tr.pass[j] = (dfr >= lo) && (dfr <= hi) && (disc > 0.f);
        // disc <= 0: below the curve's minimum, command its vertex
        rc[j] = disc > 0.f ? 2.f * df * rcp_hw(sqrt_hw(disc) + P.k1w) : P.vtx;
    }
}

// VJP of allocate: wb += (d rc / d wrench)^T rcb, with d xi / d f = 1 / sqrt(disc)
__device__ __forceinline__ void allocate_vjp(const PidParams& C, const PidTrace& tr, const float* rcb, float* wb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float fb = tr.pass[j] ? rcb[j] * rsqrt_hw(tr.disc[j]) : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) wb[i] += C.A[4 * j + i] * fb;
    }
}

// Position interface: geometric controller on SO(3) (command [x, y, z, yaw]):
//   a = -kp (p - p_sp) - kv v + g e_z, F = m a, T = F . R e_z,
//   z_d = F / |F|, y_d = z_d x [cos yaw, sin yaw, 0] normalised, x_d = y_d x z_d,
//   e_R = vee(R_d^T R - R^T R_d) / 2, tau = J_ctrl (-kR e_R - kw w),
// then the allocation. The trace keeps what the VJP needs.
struct PosTrace {
    float F[3], inv_nF, zd[3], inv_ny, yd[3], xd[3], R[9], s, c;
};

__device__ __forceinline__ void pos_forward(const float* x, const float* u, const FpParams& P, const PidParams& C,
                                            float* rc, PidTrace& tr, PosTrace& pt) {
#pragma unroll
    for (int i = 0; i < 3; ++i) pt.F[i] = C.m * (-C.pkp[i] * (x[i] - u[i]) - C.pkv[i] * x[7 + i] + (i == 2 ? C.g : 0.f));
    quat_matrix(x[3], x[4], x[5], x[6], pt.R);
    const float* R = pt.R;
    const float T = pt.F[0] * R[2] + pt.F[1] * R[5] + pt.F[2] * R[8];
    pt.inv_nF = rsqrt_hw(pt.F[0] * pt.F[0] + pt.F[1] * pt.F[1] + pt.F[2] * pt.F[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) pt.zd[i] = pt.F[i] * pt.inv_nF;
    sincos_cw(u[3], &pt.s, &pt.c);
    // y = z_d x (c, s, 0)
    const float yr[3] = {-pt.zd[2] * pt.s, pt.zd[2] * pt.c, pt.zd[0] * pt.s - pt.zd[1] * pt.c};
    pt.inv_ny = rsqrt_hw(yr[0] * yr[0] + yr[1] * yr[1] + yr[2] * yr[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) pt.yd[i] = yr[i] * pt.inv_ny;
    pt.xd[0] = pt.yd[1] * pt.zd[2] - pt.yd[2] * pt.zd[1];
    pt.xd[1] = pt.yd[2] * pt.zd[0] - pt.yd[0] * pt.zd[2];
    pt.xd[2] = pt.yd[0] * pt.zd[1] - pt.yd[1] * pt.zd[0];
    // columns of R: c0 = (R0, R3, R6), c1 = (R1, R4, R7), c2 = (R2, R5, R8)
    const float e0 = 0.5f * ((pt.zd[0] * R[1] + pt.zd[1] * R[4] + pt.zd[2] * R[7]) -
                             (R[2] * pt.yd[0] + R[5] * pt.yd[1] + R[8] * pt.yd[2]));
    const float e1 = 0.5f * ((pt.xd[0] * R[2] + pt.xd[1] * R[5] + pt.xd[2] * R[8]) -
                             (R[0] * pt.zd[0] + R[3] * pt.zd[1] + R[6] * pt.zd[2]));
    const float e2 = 0.5f * ((pt.yd[0] * R[0] + pt.yd[1] * R[3] + pt.yd[2] * R[6]) -
                             (R[1] * pt.xd[0] + R[4] * pt.xd[1] + R[7] * pt.xd[2]));
    const float eR[3] = {e0, e1, e2};
    float wrench[4];
    wrench[0] = T;
#pragma unroll
    for (int i = 0; i < 3; ++i) wrench[1 + i] = C.jc[i] * (-C.akr[i] * eR[i] - C.akw[i] * x[10 + i]);
    allocate(wrench, P, C, rc, tr);
}

// xb (state, rows 0..12) and ub accumulate (d rc / d (x, u))^T rcb
__device__ __forceinline__ void pos_vjp(const float* x, const PidParams& C, const PidTrace& tr, const PosTrace& pt,
                                        const float* rcb, float* xb, float* ub) {
    float wb[4] = {0.f, 0.f, 0.f, 0.f};
    allocate_vjp(C, tr, rcb, wb);
    const float Tb = wb[0];
    float eb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        eb[i] = -0.5f * C.jc[i] * C.akr[i] * wb[1 + i];   // includes the 1/2 of e_R
        xb[10 + i] -= C.jc[i] * C.akw[i] * wb[1 + i];
    }
    const float* R = pt.R;
    const float c0[3] = {R[0], R[3], R[6]}, c1[3] = {R[1], R[4], R[7]}, c2[3] = {R[2], R[5], R[8]};
    float c0b[3], c1b[3], c2b[3], zdb[3], ydb[3], xdb[3], Fb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // e0 = (zd . c1 - c2 . yd)/2, e1 = (xd . c2 - c0 . zd)/2, e2 = (yd . c0 - c1 . xd)/2
        zdb[i] = eb[0] * c1[i] - eb[1] * c0[i];
        ydb[i] = -eb[0] * c2[i] + eb[2] * c0[i];
        xdb[i] = eb[1] * c2[i] - eb[2] * c1[i];
        c0b[i] = -eb[1] * pt.zd[i] + eb[2] * pt.yd[i];
        c1b[i] = eb[0] * pt.zd[i] - eb[2] * pt.xd[i];
        c2b[i] = -eb[0] * pt.yd[i] + eb[1] * pt.xd[i] + Tb * pt.F[i];   // T = F . c2
        Fb[i] = Tb * c2[i];
    }
    // xd = yd x zd
    ydb[0] += pt.zd[1] * xdb[2] - pt.zd[2] * xdb[1];
    ydb[1] += pt.zd[2] * xdb[0] - pt.zd[0] * xdb[2];
    ydb[2] += pt.zd[0] * xdb[1] - pt.zd[1] * xdb[0];
    zdb[0] += xdb[1] * pt.yd[2] - xdb[2] * pt.yd[1];
    zdb[1] += xdb[2] * pt.yd[0] - xdb[0] * pt.yd[2];
    zdb[2] += xdb[0] * pt.yd[1] - xdb[1] * pt.yd[0];
    // yd = y / |y|
    const float dy = pt.yd[0] * ydb[0] + pt.yd[1] * ydb[1] + pt.yd[2] * ydb[2];
    float yb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) yb[i] = (ydb[i] - pt.yd[i] * dy) * pt.inv_ny;
    // y = zd x xc, xc = (c, s, 0)
    zdb[0] += pt.s * yb[2];                       // (xc x yb)_0 = s yb2 - 0 yb1
    zdb[1] += -pt.c * yb[2];                      // (xc x yb)_1 = 0 yb0 - c yb2
    zdb[2] += pt.c * yb[1] - pt.s * yb[0];        // (xc x yb)_2
    const float xcb0 = yb[1] * pt.zd[2] - yb[2] * pt.zd[1];
    const float xcb1 = yb[2] * pt.zd[0] - yb[0] * pt.zd[2];
    ub[3] += -pt.s * xcb0 + pt.c * xcb1;
    // zd = F / |F|
    const float dz = pt.zd[0] * zdb[0] + pt.zd[1] * zdb[1] + pt.zd[2] * zdb[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) Fb[i] += (zdb[i] - pt.zd[i] * dz) * pt.inv_nF;
    // F = m (-kp (p - p_sp) - kv v + g e_z)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float ab = C.m * Fb[i];
        xb[i] -= C.pkp[i] * ab;
        ub[i] += C.pkp[i] * ab;
        xb[7 + i] -= C.pkv[i] * ab;
    }
    float Rb[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Rb[3 * i] = c0b[i];
        Rb[3 * i + 1] = c1b[i];
        Rb[3 * i + 2] = c2b[i];
    }
    quat_matrix_vjp(x[3], x[4], x[5], x[6], Rb, xb + 3);
}

// x: 25-component state; u: [roll, pitch, yawrate, thrust]. Writes rotor
// commands rc[4] and the new controller state cs[8] = [I_a(2), I_r(3), w_prev(3)].
__device__ __forceinline__ void pid_forward(const float* x, const float* u, const FpParams& P,
                                            const PidParams& C, float dt, float inv_dt,
                                            float* rc, float* cs, PidTrace& tr) {
    const float qx = x[3], qy = x[4], qz = x[5], qw = x[6];
    tr.s1 = 2.f * (qw * qx + qy * qz);
    tr.c1 = 1.f - 2.f * (qx * qx + qy * qy);
    tr.s2 = 2.f * (qw * qy - qz * qx);
    const float roll = atan2_poly(tr.s1, tr.c1);
    const float pitch = asin_poly(fminf(fmaxf(tr.s2, -1.f), 1.f));
    const float ea0 = u[0] - roll, ea1 = u[1] - pitch;
    cs[0] = x[17] + ea0 * dt;
    cs[1] = x[18] + ea1 * dt;
    float rs[3];
    rs[0] = C.akp[0] * ea0 + C.aki[0] * cs[0];
    rs[1] = C.akp[1] * ea1 + C.aki[1] * cs[1];
    rs[2] = u[2];
    float tq[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float w = x[10 + i];
        const float er = rs[i] - w;
        cs[2 + i] = x[19 + i] + er * dt;
        const float al = C.rkp[i] * er + C.rki[i] * cs[2 + i] - C.rkd[i] * (w - x[22 + i]) * inv_dt;
        tq[i] = C.jc[i] * al;
        cs[5 + i] = w;
    }
    const float wrench[4] = {u[3], tq[0], tq[1], tq[2]};
    allocate(wrench, P, C, rc, tr);
}

// VJP of pid_forward. rcb: adjoint of rc; csb: adjoint of the new controller state.
// Accumulates into xb (25) and ub (4).
__device__ __forceinline__ void pid_vjp(const float* x, const FpParams& P, const PidParams& C,
                                        float dt, float inv_dt, const PidTrace& tr,
                                        const float* rcb, const float* csb, float* xb, float* ub) {
    float wb[4] = {0.f, 0.f, 0.f, 0.f};
    allocate_vjp(C, tr, rcb, wb);
    ub[3] += wb[0];
    const float tqb[3] = {wb[1], wb[2], wb[3]};
    float rsb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float alb = C.jc[i] * tqb[i];
        const float irb = csb[2 + i] + C.rki[i] * alb;   // adjoint of the updated integral
        xb[19 + i] += irb;
        const float erb = C.rkp[i] * alb + irb * dt;
        const float dterm = C.rkd[i] * alb * inv_dt;
        xb[10 + i] += -erb - dterm + csb[5 + i];
        xb[22 + i] += dterm;
        rsb[i] = erb;
    }
    ub[2] += rsb[2];
    float eab[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float iab = csb[j] + C.aki[j] * rsb[j];
        xb[17 + j] += iab;
        eab[j] = C.akp[j] * rsb[j] + iab * dt;
    }
    ub[0] += eab[0];
    ub[1] += eab[1];
    const float rollb = -eab[0], pitchb = -eab[1];
    const float iden = rcp_hw(tr.s1 * tr.s1 + tr.c1 * tr.c1);
    const float s1b = rollb * tr.c1 * iden;
    const float c1b = -rollb * tr.s1 * iden;
    const float s2b = (tr.s2 >= -1.f && tr.s2 <= 1.f) ? pitchb * rsqrt_hw(1.f - tr.s2 * tr.s2) : 0.f;
    const float qx = x[3], qy = x[4], qz = x[5], qw = x[6];
    xb[3] += 2.f * qw * s1b - 4.f * qx * c1b - 2.f * qz * s2b;
    xb[4] += 2.f * qz * s1b - 4.f * qy * c1b + 2.f * qw * s2b;
    xb[5] += 2.f * qy * s1b - 2.f * qx * s2b;
    xb[6] += 2.f * qx * s1b + 2.f * qy * s2b;
}

// ---------------------------------------------------------------------------
// integrators over an N-component state with a rates functor rates(xin, xdot).
// Rows set in MASK take the final update x += d with compensated (Kahan)
// summation; c[] carries each row's lost low-order part from step to step while
// the state stays in registers (rotor speeds ~1e4 and growing positions and
// velocities would otherwise drop increments below half an FP32 ulp).
// rates1 evaluates the first stage (at x itself), rates the others
template <int N, int INTEG, uint32_t MASK, class Rates1, class Rates>
__device__ __forceinline__ void integrate(float* x, float* c, float h, const Rates1& rates1, const Rates& rates) {
    float k[N], d[N];
    if constexpr (INTEG == EULER) {
        rates1(x, k);
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = h * k[i];
    } else {
        float acc[N], xs[N];
        const float h2 = 0.5f * h, h6 = h * (1.0f / 6.0f);
        rates1(x, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { acc[i] = k[i]; xs[i] = x[i] + h2 * k[i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { acc[i] += 2.f * k[i]; xs[i] = x[i] + h2 * k[i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { acc[i] += 2.f * k[i]; xs[i] = x[i] + h * k[i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = h6 * (acc[i] + k[i]);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if ((MASK >> i) & 1u) {
            const float y = d[i] - c[i];
            const float t = x[i] + y;
            c[i] = (t - x[i]) - y;
            x[i] = t;
        } else {
            x[i] += d[i];
        }
    }
}

template <int N, int INTEG, uint32_t MASK, class Rates>
__device__ __forceinline__ void integrate(float* x, float* c, float h, const Rates& rates) {
    integrate<N, INTEG, MASK>(x, c, h, rates, rates);
}

// The first-principles step when the rotor law is W' = c_v (W_cmd - W) (no
// quadratic term, one coefficient on both branches, no rotor inertia): with the
// command held over the step the four rotor rows form a linear system of their
// own, so their RK4 stage values and update are polynomials in z = c_v h applied
// to e0 = W - W_cmd (the same numbers RK4 produces, without its per-row
// bookkeeping):
//   stage 2: W_cmd + e0 (1 - z/2), stage 3: W_cmd + e0 (1 - z/2 + z^2/4),
//   stage 4: W_cmd + e0 (1 - z + z^2/2 - z^3/4),
//   update:  W_cmd + e0 (1 - z + z^2/2 - z^3/6 + z^4/24);
// Euler: W_cmd + e0 (1 - z). The rigid-body rows 0..12 integrate as in
// integrate(), with the rotor rates of the rates function left unused.
template <int INTEG, uint32_t MASK, class Rates>
__device__ __forceinline__ void integrate_fp_linear_rotors(float* x, float* c, float h, const float* rc, float cv,
                                                           const Rates& rates) {
    constexpr int NB = 13;   // rigid-body rows
    const float z = cv * h;
    float e0[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e0[i] = x[13 + i] - rc[i];
    float k[S_FP], d[NB];
    if constexpr (INTEG == EULER) {
        rates(x, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) d[i] = h * k[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[13 + i] = __builtin_fmaf(e0[i], 1.f - z, rc[i]);
    } else {
        const float z2 = z * z;
        const float p2 = __builtin_fmaf(-0.5f, z, 1.f);
        const float p3 = __builtin_fmaf(0.25f, z2, p2);
        const float p4 = __builtin_fmaf(z2, __builtin_fmaf(-0.25f, z, 0.5f), 1.f - z);
        const float pf = __builtin_fmaf(z2, __builtin_fmaf(z, __builtin_fmaf(z, 1.f / 24.f, -1.f / 6.f), 0.5f), 1.f - z);
        float acc[NB], xs[S_FP];
        const float h2 = 0.5f * h, h6 = h * (1.0f / 6.0f);
        rates(x, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) { acc[i] = k[i]; xs[i] = x[i] + h2 * k[i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) xs[13 + i] = __builtin_fmaf(e0[i], p2, rc[i]);
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) { acc[i] += 2.f * k[i]; xs[i] = x[i] + h2 * k[i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) xs[13 + i] = __builtin_fmaf(e0[i], p3, rc[i]);
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) { acc[i] += 2.f * k[i]; xs[i] = x[i] + h * k[i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) xs[13 + i] = __builtin_fmaf(e0[i], p4, rc[i]);
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) d[i] = h6 * (acc[i] + k[i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[13 + i] = __builtin_fmaf(e0[i], pf, rc[i]);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if ((MASK >> i) & 1u) {
            const float y = d[i] - c[i];
            const float t = x[i] + y;
            c[i] = (t - x[i]) - y;
            x[i] = t;
        } else {
            x[i] += d[i];
        }
    }
}

// rows with compensated updates: position, velocity (both models; the rotor
// rows hold deviations from the reference speed, whose increments are not lost)
constexpr uint32_t COMP_FP = 0x7u | (0x7u << 7);
constexpr uint32_t COMP_ID = 0x7u | (0x7u << 6);
constexpr uint32_t COMP_NONE = 0u;

// VJP of one integration step y = Phi(x) with the command held.
// yb: adjoint of the step's output. post(y, yb) may rewrite yb using the
// integrator output y before the reverse sweep (the renormalisation that
// follows the step); it receives y only when NEED_Y. Writes
// xb = (dPhi/dx)^T yb; vjp(xin, gb, xa) adds (d rates/d xin)^T gb into xa and
// accumulates the command adjoint itself.
// rates1 / vjp1 serve the first stage (at x itself), rates / vjp the others
template <int N, int INTEG, bool NEED_Y, class Rates, class Vjp, class Post, class Rates1, class Vjp1>
__device__ __forceinline__ void integrate_vjp(const float* x, float h, const float* yb_in, float* xb,
                                              const Rates& rates, const Vjp& vjp, const Post& post,
                                              const Rates1& rates1, const Vjp1& vjp1) {
    float yb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) yb[i] = yb_in[i];
    if constexpr (INTEG == EULER) {
        if constexpr (NEED_Y) {
            float k[N], y[N];
            rates1(x, k);
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = x[i] + h * k[i];
            post(y, yb);
        }
        float gb[N];
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] = yb[i]; gb[i] = h * yb[i]; }
        vjp1(x, gb, xb);
    } else {
        const float h2 = 0.5f * h;
        float xs[N], k[N], acc[N], x2[N], x3[N];   // stage states 2 and 3 kept for the reverse sweep
        rates1(x, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { xs[i] = x[i] + h2 * k[i]; acc[i] = k[i]; x2[i] = xs[i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { xs[i] = x[i] + h2 * k[i]; acc[i] += 2.f * k[i]; x3[i] = xs[i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { xs[i] = x[i] + h * k[i]; acc[i] += 2.f * k[i]; }
        const float h6 = h * (1.0f / 6.0f), h3 = h * (1.0f / 3.0f);
        if constexpr (NEED_Y) {
            rates(xs, k);
            float y[N];
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = x[i] + h6 * (acc[i] + k[i]);
            post(y, yb);
        }
        // reverse sweep: kb4 = h/6 yb, kb3 = h/3 yb + h a4, kb2 = h/3 yb + h/2 a3,
        // kb1 = h/6 yb + h/2 a2, with a_s = (d k_s / d x_s)^T kb_s
        float gb[N], a[N];
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] = yb[i]; gb[i] = h6 * yb[i]; a[i] = 0.f; }
        vjp(xs, gb, a);                       // stage 4 at x + h k3
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] += a[i]; gb[i] = h3 * yb[i] + h * a[i]; a[i] = 0.f; }
        vjp(x3, gb, a);                       // stage 3
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] += a[i]; gb[i] = h3 * yb[i] + h2 * a[i]; a[i] = 0.f; }
        vjp(x2, gb, a);                       // stage 2
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] += a[i]; gb[i] = h6 * yb[i] + h2 * a[i]; a[i] = 0.f; }
        vjp1(x, gb, a);                       // stage 1
#pragma unroll
        for (int i = 0; i < N; ++i) xb[i] += a[i];
    }
}

template <int N, int INTEG, bool NEED_Y, class Rates, class Vjp, class Post>
__device__ __forceinline__ void integrate_vjp(const float* x, float h, const float* yb_in, float* xb,
                                              const Rates& rates, const Vjp& vjp, const Post& post) {
    integrate_vjp<N, INTEG, NEED_Y>(x, h, yb_in, xb, rates, vjp, post, rates, vjp);
}

// VJP of integrate_fp_linear_rotors: the rigid-body rows 0..12 run the RK4
// (or Euler) reverse sweep of integrate_vjp; the rotor rows enter each stage
// through the closed form W_s = W_cmd + c_s (W - W_cmd), so the adjoint a_s that
// a stage's rates hand to its rotor values goes to W with c_s and to W_cmd with
// 1 - c_s (c = 1, 1 - z/2, 1 - z/2 + z^2/4, 1 - z + z^2/2 - z^3/4; the update
// carries the fourth-order polynomial). vjp(xin, gb, xa) receives rotor-row
// rate adjoints of zero. Writes xb rows 0..16 and accumulates rcb.
template <int INTEG, bool NEED_Y, class Rates, class Vjp, class Post>
__device__ __forceinline__ void integrate_vjp_fp_linear_rotors(const float* x, float h, const float* rc, float cv,
                                                               const float* yb_in, float* xb, float* rcb,
                                                               const Rates& rates, const Vjp& vjp, const Post& post) {
    constexpr int NB = 13;
    const float z = cv * h;
    float yb[S_FP], e0[4];
#pragma unroll
    for (int i = 0; i < S_FP; ++i) yb[i] = yb_in[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) e0[i] = x[13 + i] - rc[i];
    if constexpr (INTEG == EULER) {
        if constexpr (NEED_Y) {
            float k[S_FP], y[S_FP];
            rates(x, k);
#pragma unroll
            for (int i = 0; i < NB; ++i) y[i] = x[i] + h * k[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) y[13 + i] = __builtin_fmaf(e0[i], 1.f - z, rc[i]);
            post(y, yb);
        }
        float gb[S_FP];
#pragma unroll
        for (int i = 0; i < S_FP; ++i) { xb[i] = i < NB ? yb[i] : 0.f; gb[i] = i < NB ? h * yb[i] : 0.f; }
        vjp(x, gb, xb);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            xb[13 + i] += (1.f - z) * yb[13 + i];
            rcb[i] += z * yb[13 + i];
        }
    } else {
        const float h2 = 0.5f * h;
        const float z2 = z * z;
        const float p2 = __builtin_fmaf(-0.5f, z, 1.f);
        const float p3 = __builtin_fmaf(0.25f, z2, p2);
        const float p4 = __builtin_fmaf(z2, __builtin_fmaf(-0.25f, z, 0.5f), 1.f - z);
        const float pf = __builtin_fmaf(z2, __builtin_fmaf(z, __builtin_fmaf(z, 1.f / 24.f, -1.f / 6.f), 0.5f), 1.f - z);
        float xs[S_FP], k[S_FP], acc[NB], x2[S_FP], x3[S_FP];
        rates(x, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) { xs[i] = x[i] + h2 * k[i]; acc[i] = k[i]; x2[i] = xs[i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) { xs[13 + i] = __builtin_fmaf(e0[i], p2, rc[i]); x2[13 + i] = xs[13 + i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) { xs[i] = x[i] + h2 * k[i]; acc[i] += 2.f * k[i]; x3[i] = xs[i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) { xs[13 + i] = __builtin_fmaf(e0[i], p3, rc[i]); x3[13 + i] = xs[13 + i]; }
        rates(xs, k);
#pragma unroll
        for (int i = 0; i < NB; ++i) { xs[i] = x[i] + h * k[i]; acc[i] += 2.f * k[i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i) xs[13 + i] = __builtin_fmaf(e0[i], p4, rc[i]);
        const float h6 = h * (1.0f / 6.0f), h3 = h * (1.0f / 3.0f);
        if constexpr (NEED_Y) {
            rates(xs, k);
            float y[S_FP];
#pragma unroll
            for (int i = 0; i < NB; ++i) y[i] = x[i] + h6 * (acc[i] + k[i]);
#pragma unroll
            for (int i = 0; i < 4; ++i) y[13 + i] = __builtin_fmaf(e0[i], pf, rc[i]);
            post(y, yb);
        }
        // rigid rows: kb4 = h/6 yb, kb3 = h/3 yb + h a4, kb2 = h/3 yb + h/2 a3,
        // kb1 = h/6 yb + h/2 a2; rotor rows: W gets sum_s c_s a_s + pf yb, W_cmd
        // the remainder of sum_s a_s + yb
        float gb[S_FP], a[S_FP], wr[4], cr[4];
#pragma unroll
        for (int i = 0; i < S_FP; ++i) { gb[i] = i < NB ? h6 * yb[i] : 0.f; a[i] = 0.f; }
#pragma unroll
        for (int i = 0; i < NB; ++i) xb[i] = yb[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) { wr[i] = pf * yb[13 + i]; cr[i] = yb[13 + i]; }
        vjp(xs, gb, a);                       // stage 4 at (x + h k3, W_cmd + p4 e0)
#pragma unroll
        for (int i = 0; i < NB; ++i) { xb[i] += a[i]; gb[i] = h3 * yb[i] + h * a[i]; a[i] = 0.f; }
#pragma unroll
        for (int i = 0; i < 4; ++i) { wr[i] = __builtin_fmaf(p4, a[13 + i], wr[i]); cr[i] += a[13 + i]; a[13 + i] = 0.f; }
        vjp(x3, gb, a);                       // stage 3
#pragma unroll
        for (int i = 0; i < NB; ++i) { xb[i] += a[i]; gb[i] = h3 * yb[i] + h2 * a[i]; a[i] = 0.f; }
#pragma unroll
        for (int i = 0; i < 4; ++i) { wr[i] = __builtin_fmaf(p3, a[13 + i], wr[i]); cr[i] += a[13 + i]; a[13 + i] = 0.f; }
        vjp(x2, gb, a);                       // stage 2
#pragma unroll
        for (int i = 0; i < NB; ++i) { xb[i] += a[i]; gb[i] = h6 * yb[i] + h2 * a[i]; a[i] = 0.f; }
#pragma unroll
        for (int i = 0; i < 4; ++i) { wr[i] = __builtin_fmaf(p2, a[13 + i], wr[i]); cr[i] += a[13 + i]; a[13 + i] = 0.f; }
        vjp(x, gb, a);                        // stage 1 (c = 1: nothing for W_cmd)
#pragma unroll
        for (int i = 0; i < NB; ++i) xb[i] += a[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            xb[13 + i] = wr[i] + a[13 + i];
            rcb[i] += cr[i] - wr[i];
        }
    }
}

// ---------------------------------------------------------------------------
// whole steps

// The onboard controller of the first-principles model (attitude PID, position
// controller, torque allocation) at (x, u) with controller period dtc: rotor
// commands rc (deviations from W_r) and, for the PID, its new state cs.
template <int CTRL>
__device__ __forceinline__ void fp_ctrl_forward(const float* x, const float* u, const FpParams& P,
                                                const PidParams& C, float dtc, float inv_dtc, float* rc, float* cs) {
    PidTrace tr;
    if constexpr (CTRL == CTRL_PID) {
        pid_forward(x, u, P, C, dtc, inv_dtc, rc, cs, tr);
    } else if constexpr (CTRL == CTRL_TORQUE) {
        allocate(u, P, C, rc, tr);
    } else if constexpr (CTRL == CTRL_POSITION) {
        PosTrace pt;
        pos_forward(x, u, P, C, rc, tr, pt);
    }
}

// first-principles step; S = 17 (rotor interface) or 25 (attitude PID).
// rc holds the rotor-speed commands across steps (owned by the caller). The
// onboard controller runs when ctrl_now, with its own period dtc (a whole number
// of physics steps); in between its commands are held and the PID state is
// carried. The rotor interface applies its command every step.
template <int CTRL, int INTEG>
__device__ __forceinline__ void fp_step(float* x, float* comp, const float* u, const FpParams& P,
                                        const PidParams& C, float dt, float dtc, float inv_dtc, int renorm,
                                        float* rc, bool ctrl_now) {
    if constexpr (CTRL == CTRL_ROTOR) {
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[i] = u[i] - P.wr;
    } else {
        if (ctrl_now) {
            float cs[8];
            fp_ctrl_forward<CTRL>(x, u, P, C, dtc, inv_dtc, rc, cs);
            // the PID's new state goes to its rows at once: the integration below
            // reads and writes rows 0..16 only
            if constexpr (CTRL == CTRL_PID) {
#pragma unroll
                for (int i = 0; i < 8; ++i) x[17 + i] = cs[i];
            }
        }
    }
    if (!P.rotor_general && !P.gyro)
        integrate_fp_linear_rotors<INTEG, COMP_FP>(x, comp, dt, rc, P.cvu,
                                                   [&](const float* xi, float* xd) { fp_rates(xi, rc, P, xd); });
    else
        integrate<S_FP, INTEG, COMP_FP>(x, comp, dt, [&](const float* xi, float* xd) { fp_rates(xi, rc, P, xd); });
    if (renorm) {
        const float n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
        const float inv = rsqrt_hw(n2);
        x[3] *= inv; x[4] *= inv; x[5] *= inv; x[6] *= inv;
    }
}

// Moves the Euler-angle base to the angles a: sin and cos at a by the angle
// addition from the current base (a is one step away, so the offset is small;
// beyond 1/16 rad sincos3 takes over). Chained over a few steps the rounding
// of the recurrence grows by about one ulp per step, so callers re-anchor with
// euler_base periodically.
__device__ __forceinline__ void euler_rebase(const float* a, EulerBase& b) {
    float s[3], c[3];
    sincos3_near(a, b, s, c);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        b.a0[i] = a[i];
        b.s0[i] = s[i];
        b.c0[i] = c[i];
    }
}

// identified-model step with the Euler-angle trigonometry of the step's start
// state given in B
template <int INTEG>
__device__ __forceinline__ void id_step_base(float* x, float* comp, const float* u, const IdParams& P, float dt,
                                             const EulerBase& B) {
    integrate<S_ID, INTEG, COMP_ID>(
        x, comp, dt, [&](const float* xi, float* xd) { id_rates<true>(xi, u, P, B, xd); },
        [&](const float* xi, float* xd) { id_rates(xi, u, P, B, xd); });
    if (P.direct) x[12] = u[3];  // the thrust row holds the applied thrust
}

template <int INTEG>
__device__ __forceinline__ void id_step(float* x, float* comp, const float* u, const IdParams& P, float dt) {
    EulerBase B;
    euler_base(x + 3, B);
    integrate<S_ID, INTEG, COMP_ID>(
        x, comp, dt, [&](const float* xi, float* xd) { id_rates<true>(xi, u, P, B, xd); },
        [&](const float* xi, float* xd) { id_rates(xi, u, P, B, xd); });
    if (P.direct) x[12] = u[3];  // the thrust row holds the applied thrust
}

// adjoint of the renormalisation q_out = q / |q| that follows a step, given the
// integrator output y: qb <- (qb_out - q_out (q_out . qb_out)) / |q|
__device__ __forceinline__ void renorm_vjp(const float* y, float* ybr) {
    const float inv = rsqrt_hw(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
    const float q0 = y[3] * inv, q1 = y[4] * inv, q2 = y[5] * inv, q3 = y[6] * inv;
    const float dot = q0 * ybr[3] + q1 * ybr[4] + q2 * ybr[5] + q3 * ybr[6];
    ybr[3] = (ybr[3] - q0 * dot) * inv;
    ybr[4] = (ybr[4] - q1 * dot) * inv;
    ybr[5] = (ybr[5] - q2 * dot) * inv;
    ybr[6] = (ybr[6] - q3 * dot) * inv;
}

// fp_held_vjp: VJP of the rigid-body and rotor integration under the held
// commands rc (the step's own controller output, or commands held from an
// earlier controller step): writes xb rows 0..16 and accumulates rcb. The
// linear rotor law without gyroscopic torques takes the closed-form rotor rows
// of the forward step.
template <int INTEG>
__device__ __forceinline__ void fp_held_vjp(const float* x, const float* rc, const FpParams& P, float dt,
                                            int renorm, const float* yb, float* xb, float* rcb) {
    const auto rates = [&](const float* xi, float* xd) { fp_rates(xi, rc, P, xd); };
    const auto vjp = [&](const float* xi, const float* gb, float* xa) { fp_rates_vjp(xi, rc, P, gb, xa, rcb); };
    const auto none = [](const float*, float*) {};
    if (!P.rotor_general && !P.gyro) {
        if (renorm)
            integrate_vjp_fp_linear_rotors<INTEG, true>(x, dt, rc, P.cvu, yb, xb, rcb, rates, vjp, renorm_vjp);
        else
            integrate_vjp_fp_linear_rotors<INTEG, false>(x, dt, rc, P.cvu, yb, xb, rcb, rates, vjp, none);
    } else if (renorm) {
        integrate_vjp<S_FP, INTEG, true>(x, dt, yb, xb, rates, vjp, renorm_vjp);
    } else {
        integrate_vjp<S_FP, INTEG, false>(x, dt, yb, xb, rates, vjp, none);
    }
}

// VJP of fp_step at (x, u) with the controller evaluated in this step: yb =
// adjoint of the new state (S components), writes xb (S) and accumulates ub (4).
template <int CTRL, int INTEG>
__device__ __forceinline__ void fp_step_vjp(const float* x, const float* u, const FpParams& P,
                                            const PidParams& C, float dt, float dtc, float inv_dtc, int renorm,
                                            const float* yb, float* xb, float* ub) {
    float rc[4], cs[8];
    PidTrace tr;
    PosTrace pt;
    if constexpr (CTRL == CTRL_PID) {
        pid_forward(x, u, P, C, dtc, inv_dtc, rc, cs, tr);
    } else if constexpr (CTRL == CTRL_TORQUE) {
        allocate(u, P, C, rc, tr);
    } else if constexpr (CTRL == CTRL_POSITION) {
        pos_forward(x, u, P, C, rc, tr, pt);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[i] = u[i] - P.wr;
    }
    float rcb[4] = {0.f, 0.f, 0.f, 0.f};
    fp_held_vjp<INTEG>(x, rc, P, dt, renorm, yb, xb, rcb);
    if constexpr (CTRL == CTRL_PID) {
#pragma unroll
        for (int i = S_FP; i < S_PID; ++i) xb[i] = 0.f;
        pid_vjp(x, P, C, dtc, inv_dtc, tr, rcb, yb + S_FP, xb, ub);
    } else if constexpr (CTRL == CTRL_TORQUE) {
        allocate_vjp(C, tr, rcb, ub);
    } else if constexpr (CTRL == CTRL_POSITION) {
        pos_vjp(x, C, tr, pt, rcb, xb, ub);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) ub[i] += rcb[i];
    }
}

// Reverse piece of a step whose controller runs every n > 1 physics steps.
// fp_ctrl_vjp: VJP of one controller evaluation at (x, u), given the adjoint rcb
// of its held commands (summed over the steps that used them) and csb of the PID
// state it wrote (rows 17..24 of the next state): accumulates into xb and ub.
template <int CTRL>
__device__ __forceinline__ void fp_ctrl_vjp(const float* x, const float* u, const FpParams& P,
                                            const PidParams& C, float dtc, float inv_dtc, const float* rcb,
                                            const float* csb, float* xb, float* ub) {
    float rc[4];
    PidTrace tr;
    if constexpr (CTRL == CTRL_PID) {
        float cs[8];
        pid_forward(x, u, P, C, dtc, inv_dtc, rc, cs, tr);
        pid_vjp(x, P, C, dtc, inv_dtc, tr, rcb, csb, xb, ub);
    } else if constexpr (CTRL == CTRL_TORQUE) {
        allocate(u, P, C, rc, tr);
        allocate_vjp(C, tr, rcb, ub);
    } else if constexpr (CTRL == CTRL_POSITION) {
        PosTrace pt;
        pos_forward(x, u, P, C, rc, tr, pt);
        pos_vjp(x, C, tr, pt, rcb, xb, ub);
    }
}

template <int INTEG>
__device__ __forceinline__ void id_step_vjp(const float* x, const float* u, const IdParams& P, float dt,
                                            const float* yb, float* xb, float* ub) {
    float ym[S_ID];
#pragma unroll
    for (int i = 0; i < S_ID; ++i) ym[i] = yb[i];
    if (P.direct) {  // y[12] = u[3]; the input thrust row is not used
        ub[3] += ym[12];
        ym[12] = 0.f;
    }
    EulerBase B;
    euler_base(x + 3, B);
    integrate_vjp<S_ID, INTEG, false>(
        x, dt, ym, xb,
        [&](const float* xi, float* xd) { id_rates(xi, u, P, B, xd); },
        [&](const float* xi, const float* gb, float* xa) { id_rates_vjp(xi, u, P, B, gb, xa, ub); },
        [](const float*, float*) {},
        [&](const float* xi, float* xd) { id_rates<true>(xi, u, P, B, xd); },
        [&](const float* xi, const float* gb, float* xa) { id_rates_vjp<true>(xi, u, P, B, gb, xa, ub); });
}

}  // namespace cfk
