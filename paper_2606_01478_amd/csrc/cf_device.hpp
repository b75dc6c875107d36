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

namespace cfk {

// ---------------------------------------------------------------------------
// parameter record offsets (public layout, see include/cfsim.h)
enum : int {
    P_MASS = 0, P_GRAVITY = 1, P_J = 2, P_THRUST = 5, P_TORQUE = 8, P_MIX_TX = 11,
    P_MIX_TY = 15, P_MIX_YAW = 19, P_MOTOR_UP = 23, P_MOTOR_DOWN = 25, P_JP = 27,
    P_DRAG = 28, P_ANG_KP = 31, P_ANG_KI = 33, P_RATE_KP = 35, P_RATE_KI = 38,
    P_RATE_KD = 41, P_J_CTRL = 44, P_F_MAX = 47, P_ALLOC = 48, P_CF = 64, P_CTAU = 65,
    P_CPSI1 = 66, P_CPSI2 = 69, P_CPSI3 = 72, NPARAM = 96
};
enum : int { MODEL_FP = 0, MODEL_ID = 1 };
enum : int { CTRL_ROTOR = 0, CTRL_PID = 1 };
enum : int { EULER = 0, RK4 = 1 };
constexpr int S_FP = 17, S_PID = 25, S_ID = 13;

// accessor over one world's record: array-of-structs (uniform world per tile)
struct AosRec {
    const float* r;
    __device__ __forceinline__ float operator()(int i) const { return r[i]; }
};
// accessor over a world's record in the transposed [NPARAM][M] copy (per-lane world)
struct SoaRec {
    const float* p; int M; int w;
    __device__ __forceinline__ float operator()(int i) const { return p[(size_t)i * M + w]; }
};

struct FpParams {
    float inv_m, g;
    float iJx, iJy, iJz, dJx, dJy, dJz;  // dJx = Jz - Jy, dJy = Jx - Jz, dJz = Jy - Jx
    float k0, k1, k2, t0, t1, t2, inv_2k2;
    float tx[4], ty[4], tz[4];
    float cvu, cdu, cvd, cdd;
};
struct PidParams {
    float akp[2], aki[2], rkp[3], rki[3], rkd[3], jc[3], fmax;
    float A[16];
};
struct IdParams {
    float cf_m, g, ctau, f_hover;
    float c1[3], c2[3], c3[3];
};

template <class R>
__device__ __forceinline__ FpParams load_fp(const R& rec) {
    FpParams P;
    P.inv_m = 1.0f / rec(P_MASS);
    P.g = rec(P_GRAVITY);
    const float Jx = rec(P_J), Jy = rec(P_J + 1), Jz = rec(P_J + 2);
    P.iJx = 1.0f / Jx; P.iJy = 1.0f / Jy; P.iJz = 1.0f / Jz;
    P.dJx = Jz - Jy; P.dJy = Jx - Jz; P.dJz = Jy - Jx;
    P.k0 = rec(P_THRUST); P.k1 = rec(P_THRUST + 1); P.k2 = rec(P_THRUST + 2);
    P.inv_2k2 = 0.5f / P.k2;
    P.t0 = rec(P_TORQUE); P.t1 = rec(P_TORQUE + 1); P.t2 = rec(P_TORQUE + 2);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        P.tx[i] = rec(P_MIX_TX + i); P.ty[i] = rec(P_MIX_TY + i); P.tz[i] = rec(P_MIX_YAW + i);
    }
    P.cvu = rec(P_MOTOR_UP); P.cdu = rec(P_MOTOR_UP + 1);
    P.cvd = rec(P_MOTOR_DOWN); P.cdd = rec(P_MOTOR_DOWN + 1);
    return P;
}

template <class R>
__device__ __forceinline__ PidParams load_pid(const R& rec) {
    PidParams C;
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

template <class R>
__device__ __forceinline__ IdParams load_id(const R& rec) {
    IdParams P;
    const float m = rec(P_MASS), cf = rec(P_CF);
    P.cf_m = cf / m;
    P.g = rec(P_GRAVITY);
    P.ctau = rec(P_CTAU);
    P.f_hover = m * P.g / cf;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        P.c1[i] = rec(P_CPSI1 + i); P.c2[i] = rec(P_CPSI2 + i); P.c3[i] = rec(P_CPSI3 + i);
    }
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

// hardware square root and reciprocal square root (within 1 ulp on gfx950)
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsqrt_hw(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// first-principles right-hand side, 17 components [p q v w Omega]
__device__ __forceinline__ void fp_rates(const float* x, const float* rc, const FpParams& P, float* xd) {
    const float qx = x[3], qy = x[4], qz = x[5], qw = x[6];
    const float wx = x[10], wy = x[11], wz = x[12];
    float F = 0.f, tx = 0.f, ty = 0.f, tz = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = x[13 + i];
        const bool up = rc[i] >= r;          // accelerating branch (ties included)
        const float cv = up ? P.cvu : P.cvd;
        const float cd = up ? P.cdu : P.cdd;
        xd[13 + i] = cv * (rc[i] - r) + cd * (rc[i] * rc[i] - r * r);
        const float f = P.k0 + r * (P.k1 + P.k2 * r);
        const float tq = P.t0 + r * (P.t1 + P.t2 * r);
        F += f;
        tx += P.tx[i] * f;
        ty += P.ty[i] * f;
        tz += P.tz[i] * tq;
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
    xd[10] = (tx - P.dJx * wy * wz) * P.iJx;
    xd[11] = (ty - P.dJy * wz * wx) * P.iJy;
    xd[12] = (tz - P.dJz * wx * wy) * P.iJz;
}

// VJP of fp_rates at (x, rc): xb += (d xd/d x)^T gb, rcb += (d xd/d rc)^T gb
__device__ __forceinline__ void fp_rates_vjp(const float* x, const float* rc, const FpParams& P,
                                             const float* gb, float* xb, float* rcb) {
    const float qx = x[3], qy = x[4], qz = x[5], qw = x[6];
    const float wx = x[10], wy = x[11], wz = x[12];
    float F = 0.f;
    float f[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = x[13 + i];
        f[i] = P.k0 + r * (P.k1 + P.k2 * r);
        F += f[i];
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
    // w' = (tau - w x J w) / J
    const float hx = gb[10] * P.iJx, hy = gb[11] * P.iJy, hz = gb[12] * P.iJz;
    xb[10] -= hy * P.dJy * wz + hz * P.dJz * wy;
    xb[11] -= hx * P.dJx * wz + hz * P.dJz * wx;
    xb[12] -= hx * P.dJx * wy + hy * P.dJy * wx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float r = x[13 + i];
        const float fb = Fb + P.tx[i] * hx + P.ty[i] * hy;
        const float tqb = P.tz[i] * hz;
        const bool up = rc[i] >= r;
        const float cv = up ? P.cvu : P.cvd;
        const float cd = up ? P.cdu : P.cdd;
        const float gr = gb[13 + i];
        xb[13 + i] += fb * (P.k1 + 2.f * P.k2 * r) + tqb * (P.t1 + 2.f * P.t2 * r)
                      - gr * (cv + 2.f * cd * r);
        rcb[i] += gr * (cv + 2.f * cd * rc[i]);
    }
}

// ---------------------------------------------------------------------------
// identified model right-hand side, 13 components [p Psi v dPsi f]
__device__ __forceinline__ void id_rates(const float* x, const float* u, const IdParams& P, float* xd) {
    float sn[3], cs[3];
    sincos3(x + 3, sn, cs);
    const float sph = sn[0], cph = cs[0], sth = sn[1], cth = cs[1], sps = sn[2], cps = cs[2];
    const float a = P.cf_m * x[12];
    xd[0] = x[6]; xd[1] = x[7]; xd[2] = x[8];
    xd[3] = x[9]; xd[4] = x[10]; xd[5] = x[11];
    xd[6] = a * (cps * sth * cph + sps * sph);
    xd[7] = a * (sps * sth * cph - cps * sph);
    xd[8] = a * (cth * cph) - P.g;
#pragma unroll
    for (int i = 0; i < 3; ++i) xd[9 + i] = P.c1[i] * x[3 + i] + P.c2[i] * x[9 + i] + P.c3[i] * u[i];
    xd[12] = P.ctau * (u[3] - x[12]);
}

__device__ __forceinline__ void id_rates_vjp(const float* x, const float* u, const IdParams& P,
                                             const float* gb, float* xb, float* ub) {
    float sn[3], cs[3];
    sincos3(x + 3, sn, cs);
    const float sph = sn[0], cph = cs[0], sth = sn[1], cth = cs[1], sps = sn[2], cps = cs[2];
    const float a = P.cf_m * x[12];
    const float rz0 = cps * sth * cph + sps * sph;
    const float rz1 = sps * sth * cph - cps * sph;
    const float rz2 = cth * cph;
    // p' = v, Psi' = dPsi
    xb[6] += gb[0]; xb[7] += gb[1]; xb[8] += gb[2];
    xb[9] += gb[3]; xb[10] += gb[4]; xb[11] += gb[5];
    // v' = a R e_z - g e_z
    xb[12] += (gb[6] * rz0 + gb[7] * rz1 + gb[8] * rz2) * P.cf_m;
    const float b0 = a * gb[6], b1 = a * gb[7], b2 = a * gb[8];
    xb[3] += b0 * (sps * cph - cps * sth * sph) + b1 * (-sps * sth * sph - cps * cph) + b2 * (-cth * sph);
    xb[4] += b0 * (cps * cth * cph) + b1 * (sps * cth * cph) + b2 * (-sth * cph);
    xb[5] += b0 * (cps * sph - sps * sth * cph) + b1 * (cps * sth * cph + sps * sph);
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
    float s1, c1, s2, fraw[4], disc[4];
};

__device__ __forceinline__ float rotor_root(float f, float disc, const FpParams& P) {
    return disc > 0.f ? (sqrt_hw(disc) - P.k1) * P.inv_2k2 : -P.k1 * P.inv_2k2;
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
    const float roll = atan2f(tr.s1, tr.c1);
    const float pitch = asinf(fminf(fmaxf(tr.s2, -1.f), 1.f));
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
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float fr = C.A[4 * j] * u[3] + C.A[4 * j + 1] * tq[0] + C.A[4 * j + 2] * tq[1] + C.A[4 * j + 3] * tq[2];
        tr.fraw[j] = fr;
        const float f = fminf(fmaxf(fr, 0.f), C.fmax);
        tr.disc[j] = P.k1 * P.k1 - 4.f * P.k2 * (P.k0 - f);
        rc[j] = rotor_root(f, tr.disc[j], P);
    }
}

// VJP of pid_forward. rcb: adjoint of rc; csb: adjoint of the new controller state.
// Accumulates into xb (25) and ub (4).
__device__ __forceinline__ void pid_vjp(const float* x, const FpParams& P, const PidParams& C,
                                        float dt, float inv_dt, const PidTrace& tr,
                                        const float* rcb, const float* csb, float* xb, float* ub) {
    float tqb[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float fr = tr.fraw[j];
        const bool pass = (fr >= 0.f) && (fr <= C.fmax) && (tr.disc[j] > 0.f);
        const float fb = pass ? rcb[j] * rsqrt_hw(tr.disc[j]) : 0.f;
        ub[3] += C.A[4 * j] * fb;
        tqb[0] += C.A[4 * j + 1] * fb;
        tqb[1] += C.A[4 * j + 2] * fb;
        tqb[2] += C.A[4 * j + 3] * fb;
    }
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
template <int N, int INTEG, uint32_t MASK, class Rates>
__device__ __forceinline__ void integrate(float* x, float* c, float h, const Rates& rates) {
    float k[N], d[N];
    if constexpr (INTEG == EULER) {
        rates(x, k);
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = h * k[i];
    } else {
        float acc[N], xs[N];
        const float h2 = 0.5f * h, h6 = h * (1.0f / 6.0f);
        rates(x, k);
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

// rows with compensated updates: position, velocity, rotor speeds (first
// principles); position, velocity (identified)
constexpr uint32_t COMP_FP = 0x7u | (0x7u << 7) | (0xFu << 13);
constexpr uint32_t COMP_ID = 0x7u | (0x7u << 6);
constexpr uint32_t COMP_NONE = 0u;

// VJP of one integration step y = Phi(x) with the command held.
// yb: adjoint of the step's output. post(y, yb) may rewrite yb using the
// integrator output y before the reverse sweep (the renormalisation that
// follows the step); it receives y only when NEED_Y. Writes
// xb = (dPhi/dx)^T yb; vjp(xin, gb, xa) adds (d rates/d xin)^T gb into xa and
// accumulates the command adjoint itself.
template <int N, int INTEG, bool NEED_Y, class Rates, class Vjp, class Post>
__device__ __forceinline__ void integrate_vjp(const float* x, float h, const float* yb_in, float* xb,
                                              const Rates& rates, const Vjp& vjp, const Post& post) {
    float yb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) yb[i] = yb_in[i];
    if constexpr (INTEG == EULER) {
        if constexpr (NEED_Y) {
            float k[N], y[N];
            rates(x, k);
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] = x[i] + h * k[i];
            post(y, yb);
        }
        float gb[N];
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] = yb[i]; gb[i] = h * yb[i]; }
        vjp(x, gb, xb);
    } else {
        const float h2 = 0.5f * h;
        float x2[N], x3[N], x4[N], k[N];
        rates(x, k);
        float acc[N];
#pragma unroll
        for (int i = 0; i < N; ++i) { x2[i] = x[i] + h2 * k[i]; acc[i] = k[i]; }
        rates(x2, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { x3[i] = x[i] + h2 * k[i]; acc[i] += 2.f * k[i]; }
        rates(x3, k);
#pragma unroll
        for (int i = 0; i < N; ++i) { x4[i] = x[i] + h * k[i]; acc[i] += 2.f * k[i]; }
        const float h6 = h * (1.0f / 6.0f), h3 = h * (1.0f / 3.0f);
        if constexpr (NEED_Y) {
            rates(x4, k);
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
        vjp(x4, gb, a);
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] += a[i]; gb[i] = h3 * yb[i] + h * a[i]; a[i] = 0.f; }
        vjp(x3, gb, a);
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] += a[i]; gb[i] = h3 * yb[i] + h2 * a[i]; a[i] = 0.f; }
        vjp(x2, gb, a);
#pragma unroll
        for (int i = 0; i < N; ++i) { xb[i] += a[i]; gb[i] = h6 * yb[i] + h2 * a[i]; a[i] = 0.f; }
        vjp(x, gb, a);
#pragma unroll
        for (int i = 0; i < N; ++i) xb[i] += a[i];
    }
}

// ---------------------------------------------------------------------------
// whole steps

// first-principles step; S = 17 (rotor interface) or 25 (attitude PID)
template <int CTRL, int INTEG>
__device__ __forceinline__ void fp_step(float* x, float* comp, const float* u, const FpParams& P,
                                        const PidParams& C, float dt, float inv_dt, int renorm) {
    float rc[4];
    float cs[8];
    if constexpr (CTRL == CTRL_PID) {
        PidTrace tr;
        pid_forward(x, u, P, C, dt, inv_dt, rc, cs, tr);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[i] = u[i];
    }
    integrate<S_FP, INTEG, COMP_FP>(x, comp, dt, [&](const float* xi, float* xd) { fp_rates(xi, rc, P, xd); });
    if (renorm) {
        const float n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
        const float inv = rsqrt_hw(n2);
        x[3] *= inv; x[4] *= inv; x[5] *= inv; x[6] *= inv;
    }
    if constexpr (CTRL == CTRL_PID) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[17 + i] = cs[i];
    }
}

template <int INTEG>
__device__ __forceinline__ void id_step(float* x, float* comp, const float* u, const IdParams& P, float dt) {
    integrate<S_ID, INTEG, COMP_ID>(x, comp, dt, [&](const float* xi, float* xd) { id_rates(xi, u, P, xd); });
}

// VJP of fp_step at (x, u): yb = adjoint of the new state (S components),
// writes xb (S) and accumulates ub (4).
template <int CTRL, int INTEG>
__device__ __forceinline__ void fp_step_vjp(const float* x, const float* u, const FpParams& P,
                                            const PidParams& C, float dt, float inv_dt, int renorm,
                                            const float* yb, float* xb, float* ub) {
    float rc[4], cs[8];
    PidTrace tr;
    if constexpr (CTRL == CTRL_PID) {
        pid_forward(x, u, P, C, dt, inv_dt, rc, cs, tr);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) rc[i] = u[i];
    }
    float rcb[4] = {0.f, 0.f, 0.f, 0.f};
    const auto rates = [&](const float* xi, float* xd) { fp_rates(xi, rc, P, xd); };
    const auto vjp = [&](const float* xi, const float* gb, float* xa) { fp_rates_vjp(xi, rc, P, gb, xa, rcb); };
    if (renorm) {
        // q_out = q / |q| after the step: qb <- (qb_out - q_out (q_out . qb_out)) / |q|
        const auto post = [&](const float* y, float* ybr) {
            const float inv = rsqrt_hw(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
            const float q0 = y[3] * inv, q1 = y[4] * inv, q2 = y[5] * inv, q3 = y[6] * inv;
            const float dot = q0 * ybr[3] + q1 * ybr[4] + q2 * ybr[5] + q3 * ybr[6];
            ybr[3] = (ybr[3] - q0 * dot) * inv;
            ybr[4] = (ybr[4] - q1 * dot) * inv;
            ybr[5] = (ybr[5] - q2 * dot) * inv;
            ybr[6] = (ybr[6] - q3 * dot) * inv;
        };
        integrate_vjp<S_FP, INTEG, true>(x, dt, yb, xb, rates, vjp, post);
    } else {
        integrate_vjp<S_FP, INTEG, false>(x, dt, yb, xb, rates, vjp, [](const float*, float*) {});
    }
    if constexpr (CTRL == CTRL_PID) {
#pragma unroll
        for (int i = S_FP; i < S_PID; ++i) xb[i] = 0.f;
        pid_vjp(x, P, C, dt, inv_dt, tr, rcb, yb + S_FP, xb, ub);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) ub[i] += rcb[i];
    }
}

template <int INTEG>
__device__ __forceinline__ void id_step_vjp(const float* x, const float* u, const IdParams& P, float dt,
                                            const float* yb, float* xb, float* ub) {
    integrate_vjp<S_ID, INTEG, false>(
        x, dt, yb, xb,
        [&](const float* xi, float* xd) { id_rates(xi, u, P, xd); },
        [&](const float* xi, const float* gb, float* xa) { id_rates_vjp(xi, u, P, gb, xa, ub); },
        [](const float*, float*) {});
}

}  // namespace cfk
