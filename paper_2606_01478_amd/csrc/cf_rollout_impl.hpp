// Rollout kernels, shared by the forward and backward translation units
// (cf_rollout.hip, cf_rollout_bwd.hip): the forward pass with per-step
// commands, feedback (linear or the small-MLP policy), the objective and
// checkpoints; and the hand-written discrete adjoint that recomputes every
// checkpoint segment and sweeps it in reverse.
//
// Objective (per drone d, t_n = n dt):
//   u_t  = ubar_t + G_w (x_t[0:13] - x_ref(t))                (feedback, optional)
//   loss = sum_{t=1..T} |p_t - p_ref(t)|^2 + w_u sum_{t=0..T-1} |u_t|^2
// Adjoint: lambda_T = 0; for t = T-1..0:
//   lambda_{t+1} += 2 dloss (p_{t+1} - p_ref(t+1))
//   (xbar, ubar) = VJP of the step at (x_t, u_t) applied to lambda_{t+1}
//   ubar += 2 dloss w_u u_t;  g_cmds[t] = ubar;  xbar[0:13] += G^T ubar;
//   dL/dG += ubar e_t^T;  lambda_t = xbar.
#pragma once
#include <type_traits>

#include "cf_device.hpp"
#include "cf_internal.hpp"

namespace cfk {

constexpr int NG = 52;  // 4 x 13 gain entries

// The reference table is the same for every drone and never written while a
// rollout runs: its rows are read through the constant address space, i.e.
// with scalar loads into the wave's scalar registers.
__device__ __forceinline__ const const_float* ref_row(const RollArgs& a, int t, int stride) {
    return (const const_float*)(a.ref_tab + (size_t)t * stride);
}

// What of the reference is the drone's own: its position offset and, in the
// extended kernels, the rotation (cos, sin of w s and of 2 w s, w = 2 pi / P)
// that moves the shared figure-eight rows from time t to t + s for its time
// shift s. The lemniscate's x and y components are sinusoids of w t and 2 w t,
// so the shifted row follows from the shared row by the angle-sum identities:
// with p = A sin(w t), v = A w cos(w t),
//   A sin(w (t + s)) = p cos(w s) + (v / w) sin(w s),
//   A w cos(w (t + s)) = v cos(w s) - w p sin(w s),
// and likewise for the y component at 2 w.
struct RefLane {
    float off[3];
    float c1, s1, c2, s2;
};

template <bool EXT>
__device__ __forceinline__ RefLane ref_lane(const RollArgs& a, size_t D, size_t d) {
    RefLane r{{0.f, 0.f, 0.f}, 1.f, 0.f, 1.f, 0.f};
    if (a.has_obj && a.ref_off) {
#pragma unroll
        for (int j = 0; j < 3; ++j) r.off[j] = a.ref_off[j * D + d];
    }
    if constexpr (EXT) {
        if (a.has_obj && a.ref_shift) {
            sincosf(a.ref_w * a.ref_shift[d], &r.s1, &r.c1);
            r.c2 = r.c1 * r.c1 - r.s1 * r.s1;
            r.s2 = 2.f * r.s1 * r.c1;
        }
    }
    return r;
}

// figure-eight row t moved by the drone's time shift: p (3), v (3)
template <bool SH>
__device__ __forceinline__ void eight_row(const RollArgs& a, int t, const RefLane& rl, float* p, float* v) {
    const const_float* row = ref_row(a, t, 6);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        p[j] = row[j];
        v[j] = row[3 + j];
    }
    if constexpr (SH) {
        if (a.ref_shift) {
            const float w = a.ref_w, iw = a.ref_inv_w;
            const float px = p[0], vx = v[0], py = p[1], vy = v[1];
            p[0] = px * rl.c1 + (vx * iw) * rl.s1;
            v[0] = vx * rl.c1 - (w * px) * rl.s1;
            p[1] = py * rl.c2 + (vy * (0.5f * iw)) * rl.s2;
            v[1] = vy * rl.c2 - (2.f * w * py) * rl.s2;
        }
    }
}

// position reference at step t (figure-eight table rows are [p(3), v(3)])
template <bool SH>
__device__ __forceinline__ void ref_pos(const RollArgs& a, int t, const RefLane& rl, float* pr) {
    if (a.ref_user) {
        const const_float* row = ref_row(a, t, 13);
#pragma unroll
        for (int j = 0; j < 3; ++j) pr[j] = row[j] + rl.off[j];
        return;
    }
    float v[3];
    eight_row<SH>(a, t, rl, pr, v);
#pragma unroll
    for (int j = 0; j < 3; ++j) pr[j] += rl.off[j];
}

// 13-component reference state of a drone of model MODEL
template <int MODEL, bool SH>
__device__ __forceinline__ void ref_state(const RollArgs& a, int t, const RefLane& rl, float f_hover, float* xr) {
    if (a.ref_user) {
        const const_float* row = ref_row(a, t, 13);
#pragma unroll
        for (int j = 0; j < 13; ++j) xr[j] = row[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) xr[j] += rl.off[j];
        return;
    }
    float p[3], v[3];
    eight_row<SH>(a, t, rl, p, v);
#pragma unroll
    for (int j = 0; j < 13; ++j) xr[j] = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) xr[j] = p[j] + rl.off[j];
    if constexpr (MODEL == MODEL_FP) {
        xr[6] = 1.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) xr[7 + j] = v[j];
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) xr[6 + j] = v[j];
        xr[12] = f_hover;
    }
}

// per-step command ubar_t of drone d
__device__ __forceinline__ void load_cmd(const RollArgs& a, int t, size_t d, float* ub) {
    const size_t D = (size_t)a.D;
#pragma unroll
    for (int i = 0; i < 4; ++i) ub[i] = a.cmds[((size_t)t * 4 + i) * D + d];
}

// u += o, or u += s * tanh(o) for a squashed policy output (extended kernels):
// bounded commands, a normalised action a = tanh(o) scaled by s per component
template <bool EXT>
__device__ __forceinline__ void add_policy_output(const RollArgs& a, const float* o, float* u) {
    if constexpr (EXT) {
        if (a.squash) {
#pragma unroll
            for (int i = 0; i < 4; ++i) u[i] += a.act_s[i] * tanhf(o[i]);
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] += o[i];
}

// adjoint of the policy output from the adjoint ub of the applied command
template <bool EXT>
__device__ __forceinline__ void policy_output_vjp(const RollArgs& a, const float* o, const float* ub, float* ob) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ob[i] = ub[i];
    if constexpr (EXT) {
        if (a.squash) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float th = tanhf(o[i]);
                ob[i] = ub[i] * a.act_s[i] * (1.f - th * th);
            }
        }
    }
}

// applied command u = ubar + G e, e = x[0:13] - x_ref(t); returns e in ev
template <int MODEL, bool SH>
__device__ __forceinline__ void feedback(const RollArgs& a, const float* G, const float* x, int t, const RefLane& off,
                                         float f_hover, const float* ubar, float* u, float* ev) {
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ubar[i];
    if (G) {
        float xr[13];
        ref_state<MODEL, SH>(a, t, off, f_hover, xr);
#pragma unroll
        for (int j = 0; j < 13; ++j) ev[j] = x[j] - xr[j];
        float o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < 13; ++j) s += G[i * 13 + j] * ev[j];
            o[i] = s;
        }
        add_policy_output<SH>(a, o, u);
    }
}

// ---- small-MLP policy ----------------------------------------------------------
// o = W3 tanh(W2 tanh(W1 e + b1) + b2) + b3, one policy packed
// [W1 (H x 13) | b1 (H) | W2 (H x H) | b2 (H) | W3 (4 x H) | b3 (4)] in LDS (the
// same address for every lane: broadcast reads). A lane keeps its activations
// in its own LDS columns hc[k * ws]: h1 at k < H, h2 at H <= k < 2H, and in the
// backward dz2 at 2H <= k < 3H, dz1 at 3H <= k < 4H.
struct MlpView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    int H;
    __device__ __forceinline__ MlpView(const float* w, int H_) : H(H_) {
        W1 = w;
        b1 = W1 + 13 * H;
        W2 = b1 + H;
        b2 = W2 + H * H;
        W3 = b2 + H;
        b3 = W3 + 4 * H;
    }
};

// The small MLP with its width H a compile-time constant (HC) or a run-time
// value (HC = 0). With a constant width the inner sums unroll, so the LDS reads
// of weights and activations they need are issued together rather than one
// dependent read per multiply-add; the outer loops stay loops (code size).
template <int HC>
__device__ __forceinline__ void mlp_forward_w(const MlpView& m, const float* e, float* hc, int ws, float* o) {
    const int H = HC > 0 ? HC : m.H;
#pragma unroll 1
    for (int j = 0; j < H; ++j) {
        float z = m.b1[j];
#pragma unroll
        for (int i = 0; i < 13; ++i) z = fmaf(m.W1[j * 13 + i], e[i], z);
        hc[j * ws] = tanhf(z);
    }
#pragma unroll 1
    for (int j = 0; j < H; ++j) {
        float z = m.b2[j];
        if constexpr (HC > 0) {
#pragma unroll
            for (int k = 0; k < HC; ++k) z = fmaf(m.W2[j * HC + k], hc[k * ws], z);
        } else {
            for (int k = 0; k < H; ++k) z = fmaf(m.W2[j * H + k], hc[k * ws], z);
        }
        hc[(H + j) * ws] = tanhf(z);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float z = m.b3[r];
        if constexpr (HC > 0) {
#pragma unroll
            for (int k = 0; k < HC; ++k) z = fmaf(m.W3[r * HC + k], hc[(HC + k) * ws], z);
        } else {
            for (int k = 0; k < H; ++k) z = fmaf(m.W3[r * H + k], hc[(H + k) * ws], z);
        }
        o[r] = z;
    }
}

// VJP of the forward at the activations in hc, given the adjoint d3 of o:
// writes dz2 and dz1 to their columns and adds W1^T dz1 to eb (13)
template <int HC>
__device__ __forceinline__ void mlp_vjp_w(const MlpView& m, const float* d3, float* hc, int ws, float* eb) {
    const int H = HC > 0 ? HC : m.H;
#pragma unroll 1
    for (int k = 0; k < H; ++k) {
        float s = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) s = fmaf(m.W3[r * H + k], d3[r], s);
        const float h2 = hc[(H + k) * ws];
        hc[(2 * H + k) * ws] = s * (1.f - h2 * h2);
    }
#pragma unroll 1
    for (int k = 0; k < H; ++k) {
        float s = 0.f;
        if constexpr (HC > 0) {
#pragma unroll
            for (int j = 0; j < HC; ++j) s = fmaf(m.W2[j * HC + k], hc[(2 * HC + j) * ws], s);
        } else {
            for (int j = 0; j < H; ++j) s = fmaf(m.W2[j * H + k], hc[(2 * H + j) * ws], s);
        }
        const float h1 = hc[k * ws];
        hc[(3 * H + k) * ws] = s * (1.f - h1 * h1);
    }
#pragma unroll 1
    for (int j = 0; j < H; ++j) {
        const float dz = hc[(3 * H + j) * ws];
#pragma unroll
        for (int i = 0; i < 13; ++i) eb[i] = fmaf(m.W1[j * 13 + i], dz, eb[i]);
    }
}

__device__ __forceinline__ void mlp_forward(const MlpView& m, const float* e, float* hc, int ws, float* o) {
    switch (m.H) {
        case 16: mlp_forward_w<16>(m, e, hc, ws, o); break;
        case 32: mlp_forward_w<32>(m, e, hc, ws, o); break;
        default: mlp_forward_w<0>(m, e, hc, ws, o); break;
    }
}

__device__ __forceinline__ void mlp_vjp(const MlpView& m, const float* d3, float* hc, int ws, float* eb) {
    switch (m.H) {
        case 16: mlp_vjp_w<16>(m, d3, hc, ws, eb); break;
        case 32: mlp_vjp_w<32>(m, d3, hc, ws, eb); break;
        default: mlp_vjp_w<0>(m, d3, hc, ws, eb); break;
    }
}

// applied command through the MLP policy: u = ubar + o(e), e = x[0:13] - x_ref(t)
template <int MODEL>
__device__ __forceinline__ void feedback_mlp(const RollArgs& a, const MlpView& m, const float* x, int t,
                                             const RefLane& off, float f_hover, const float* ubar, float* u,
                                             float* ev, float* hc, int ws) {
    float xr[13], o[4];
    ref_state<MODEL, true>(a, t, off, f_hover, xr);
#pragma unroll
    for (int j = 0; j < 13; ++j) ev[j] = x[j] - xr[j];
    mlp_forward(m, ev, hc, ws, o);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ubar[i];
    add_policy_output<true>(a, o, u);
}

// the applied command of step t: linear feedback through G, or (extended kernels,
// mlp_H > 0) the MLP policy whose weights G points to
template <int MODEL, bool EXT>
__device__ __forceinline__ void apply_feedback(const RollArgs& a, const float* G, float* hc, int ws, const float* x,
                                               int t, const RefLane& off, float f_hover, const float* ubar, float* u,
                                               float* ev) {
    if constexpr (EXT) {
        if (a.mlp_H > 0) {
            feedback_mlp<MODEL>(a, MlpView(G, a.mlp_H), x, t, off, f_hover, ubar, u, ev, hc, ws);
            return;
        }
    }
    feedback<MODEL, EXT>(a, G, x, t, off, f_hover, ubar, u, ev);
}

template <int MODEL, int CTRL>
struct ModelTraits {
    static constexpr int S = MODEL == MODEL_ID ? S_ID : (CTRL == CTRL_PID ? S_PID : S_FP);
};

// per-drone parameters of either model
struct DroneParams {
    FpParams fp;
    PidParams pid;
    IdParams id;
};

// ---- the BPTT reward objective -------------------------------------------------
// hover command of the drone's interface: identified [0, 0, 0, m g / c_f];
// attitude [0, 0, 0, m g]; torque [m g, 0, 0, 0]; rotor the reference speed
template <int MODEL, int CTRL>
__device__ __forceinline__ void hover_action(const DroneParams& p, float* ah) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ah[i] = 0.f;
    if constexpr (MODEL == MODEL_ID) {
        ah[3] = p.id.f_hover;
    } else if constexpr (CTRL == CTRL_PID) {
        ah[3] = p.fp.g / p.fp.inv_m;
    } else if constexpr (CTRL == CTRL_TORQUE) {
        ah[0] = p.fp.g / p.fp.inv_m;
    } else if constexpr (CTRL == CTRL_ROTOR) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ah[i] = p.fp.wr;
    }
}

// angle between the body and world z axes from the attitude rows at[4]
// (quaternion x, y, z, w; or roll, pitch of the identified model's ZYX angles)
template <int MODEL>
__device__ __forceinline__ float tilt_of(const float* at) {
    if constexpr (MODEL == MODEL_FP) {
        const float n = sqrtf(at[0] * at[0] + at[1] * at[1]);
        const float c = sqrtf(at[2] * at[2] + at[3] * at[3]);
        return 2.f * atan2f(n, c);
    } else {
        float sf, cf, st, ct;
        sincosf(at[0], &sf, &cf);
        sincosf(at[1], &st, &ct);
        return atan2f(sqrtf(sf * sf + cf * cf * st * st), cf * ct);
    }
}

// xb (attitude rows) += g d tilt / d at; zero gradient at the kinks
template <int MODEL>
__device__ __forceinline__ void tilt_vjp(const float* at, float g, float* xb) {
    if constexpr (MODEL == MODEL_FP) {
        // tilt = 2 atan2(n, c), n = |(qx, qy)|, c = |(qz, qw)|
        const float n = sqrtf(at[0] * at[0] + at[1] * at[1]);
        const float c = sqrtf(at[2] * at[2] + at[3] * at[3]);
        const float Q = n * n + c * c;
        if (n > 0.f && c > 0.f) {
            const float gn = g * 2.f * c / (Q * n), gc = -g * 2.f * n / (Q * c);
            xb[3] += gn * at[0];
            xb[4] += gn * at[1];
            xb[5] += gc * at[2];
            xb[6] += gc * at[3];
        }
    } else {
        // tilt = atan2(S, C), S^2 + C^2 = 1: d tilt = C dS - S dC
        float sf, cf, st, ct;
        sincosf(at[0], &sf, &cf);
        sincosf(at[1], &st, &ct);
        const float S = sqrtf(sf * sf + cf * cf * st * st), C = cf * ct;
        if (S > 0.f) {
            xb[3] += g * (C * sf * cf * ct * ct / S + S * sf * ct);
            xb[4] += g * (C * cf * cf * st * ct / S + S * cf * st);
        }
    }
}

// attitude rows of a state: quaternion (FP) or roll, pitch (ID)
template <int MODEL>
__device__ __forceinline__ void attitude_rows(const float* x, float* at) {
    at[0] = x[3];
    at[1] = x[4];
    at[2] = MODEL == MODEL_FP ? x[5] : 0.f;
    at[3] = MODEL == MODEL_FP ? x[6] : 0.f;
}


template <int MODEL, int CTRL, bool AERO, class R>
__device__ __forceinline__ void load_params(const R& rec, DroneParams& p) {
    if constexpr (MODEL == MODEL_FP) {
        p.fp = load_fp<AERO>(rec);
    } else {
        p.id = load_id<AERO>(rec);
    }
}

// The onboard controller's gains, read right before each use (scalar loads of
// the world's record through a pointer the optimiser cannot hoist) so that they
// do not occupy registers through the integration and its reverse sweep.
template <int MODEL, int CTRL, class R>
__device__ __forceinline__ void controller_gains(const R& rec, DroneParams& p) {
    if constexpr (MODEL == MODEL_FP && CTRL != CTRL_ROTOR) p.pid = load_pid(laundered(rec), CTRL == CTRL_POSITION);
}

// one step; rc holds the first-principles rotor commands across steps, the
// onboard controller runs when ctrl_now
template <int MODEL, int CTRL, int INTEG>
__device__ __forceinline__ void model_step(float* x, float* comp, const float* u, const DroneParams& p,
                                           const RollArgs& a, float* rc, bool ctrl_now) {
    if constexpr (MODEL == MODEL_FP)
        fp_step<CTRL, INTEG>(x, comp, u, p.fp, p.pid, a.dt, a.dtc, a.inv_dtc, a.renorm, rc, ctrl_now);
    else
        id_step<INTEG>(x, comp, u, p.id, a.dt);
}

// VJP of a step whose controller (if any) runs every step
template <int MODEL, int CTRL, int INTEG>
__device__ __forceinline__ void model_step_vjp(const float* x, const float* u, const DroneParams& p,
                                               const RollArgs& a, const float* yb, float* xb, float* ub) {
    if constexpr (MODEL == MODEL_FP)
        fp_step_vjp<CTRL, INTEG>(x, u, p.fp, p.pid, a.dt, a.dtc, a.inv_dtc, a.renorm, yb, xb, ub);
    else
        id_step_vjp<INTEG>(x, u, p.id, a.dt, yb, xb, ub);
}

template <int N>
__device__ __forceinline__ void store_rows(float* dst, size_t D, size_t d, const float* x) {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i * D + d] = x[i];
}
template <int N>
__device__ __forceinline__ void load_rows(const float* src, size_t D, size_t d, float* x) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = src[i * D + d];
}

// states in caller-visible buffers (x0, checkpoints, trajectory, x_T) hold
// absolute rotor speeds; in registers and in the backward's segment buffer a
// first-principles drone holds their deviations from its reference speed
template <int MODEL>
__device__ __forceinline__ void to_dev(float* x, const DroneParams& p) {
    if constexpr (MODEL == MODEL_FP) rotors_to_dev(x, p.fp);
}
template <int MODEL, int N>
__device__ __forceinline__ void store_state(float* dst, size_t D, size_t d, const float* x, const DroneParams& p) {
    if constexpr (MODEL == MODEL_FP) {
        float y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = x[i];
        rotors_from_dev(y, p.fp);
        store_rows<N>(dst, D, d, y);
    } else {
        store_rows<N>(dst, D, d, x);
    }
}

// ---------------------------------------------------------------------------
// forward rollout of one drone
template <int MODEL, int CTRL, int INTEG, bool AERO, bool EXT, class R>
__device__ __forceinline__ void rollout_fwd_drone(const R& rec, const RollArgs& a, size_t d, int w, int S_h,
                                                  const float* G, float* hc, int ws) {
    constexpr int S = ModelTraits<MODEL, CTRL>::S;
    const size_t D = (size_t)a.D;
    const size_t SD = (size_t)S_h * D;
    DroneParams p;
    load_params<MODEL, CTRL, AERO>(rec, p);
    const float f_hover = (MODEL == MODEL_ID) ? p.id.f_hover : 0.f;
    float x[S], comp[S];
    load_rows<S>(a.x0, D, d, x);
    to_dev<MODEL>(x, p);
#pragma unroll
    for (int i = 0; i < S; ++i) comp[i] = 0.f;
    const RefLane off = ref_lane<EXT>(a, D, d);
    if (a.ckpt) store_state<MODEL, S>(a.ckpt, D, d, x, p);
    if (a.traj) store_state<MODEL, S>(a.traj, D, d, x, p);
    float loss = 0.f;
    float ubar[4];
    load_cmd(a, 0, d, ubar);
    float rc[4] = {0.f, 0.f, 0.f, 0.f};   // held rotor commands
    int phase = 0;                        // step within the controller period
    const bool rew = EXT && a.has_obj && a.obj_kind == 1;
    float uprev[4] = {0.f, 0.f, 0.f, 0.f};   // reward: the previous applied command
    if (rew) hover_action<MODEL, CTRL>(p, uprev);
    for (int t = 0; t < a.T; ++t) {
        float u[4], ev[13], unext[4];
        if (t + 1 < a.T) load_cmd(a, t + 1, d, unext);   // issued early, used next step
        apply_feedback<MODEL, EXT>(a, G, hc, ws, x, t, off, f_hover, ubar, u, ev);
        if (rew) {
            float ah[4];
            hover_action<MODEL, CTRL>(p, ah);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float da = u[i] - ah[i], dd = u[i] - uprev[i];
                loss += a.w_act[i] * da * da + a.w_dact[i] * dd * dd;
                uprev[i] = u[i];
            }
            // kept for the backward, which needs the neighbours of every command
            if (a.ubuf) {
#pragma unroll
                for (int i = 0; i < 4; ++i) a.ubuf[((size_t)t * 4 + i) * D + d] = u[i];
            }
        } else if (a.has_obj) {
            loss += a.w_u * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3]);
        }
        controller_gains<MODEL, CTRL>(rec, p);
        model_step<MODEL, CTRL, INTEG>(x, comp, u, p, a, rc, EXT ? phase == 0 : true);
        if constexpr (EXT) {
            if (++phase == a.ctrl_every) phase = 0;
        }
        if (a.has_obj) {
            float pr[3];
            ref_pos<EXT>(a, t + 1, off, pr);
            const float e0 = x[0] - pr[0], e1 = x[1] - pr[1], e2 = x[2] - pr[2];
            const float d2 = e0 * e0 + e1 * e1 + e2 * e2;
            if (rew) {
                float at[4];
                attitude_rows<MODEL>(x, at);
                loss += a.w_tilt * tilt_of<MODEL>(at) - expf(-2.f * sqrtf(d2));
            } else {
                loss += d2;
            }
        }
        const int tn = t + 1;
        if (a.ckpt && tn < a.T && (tn % a.K) == 0) store_state<MODEL, S>(a.ckpt + (size_t)(tn / a.K) * SD, D, d, x, p);
        if (a.traj) store_state<MODEL, S>(a.traj + (size_t)tn * SD, D, d, x, p);
#pragma unroll
        for (int i = 0; i < 4; ++i) ubar[i] = unext[i];
    }
    if (a.xT) store_state<MODEL, S>(a.xT, D, d, x, p);
    if (a.loss) a.loss[d] = loss;
    if (a.nonfinite) {
        bool bad = false;
#pragma unroll
        for (int i = 0; i < S; ++i) bad |= !isfinite(x[i]);
        if (bad) atomicOr(a.nonfinite + w, 1u);
    }
}

// The held rotor commands of the controller block starting at step tb: the
// controller evaluated at x_tb (checkpoint tb / K when tb is a checkpoint step,
// else slot tb - t0 of the current segment) under the command applied there.
template <int MODEL, int CTRL, int S>
__device__ __forceinline__ void block_commands(const RollArgs& a, const DroneParams& p, const float* G, float* hc,
                                               int ws, const RefLane& off, float f_hover, size_t D, size_t d,
                                               size_t SD, int tb, int t0, float* rc) {
    float xs[S], ubs[4], us[4], evs[13], cs[8];
    if (tb % a.K == 0) {
        load_rows<S>(a.ckpt_in + (size_t)(tb / a.K) * SD, D, d, xs);
        to_dev<MODEL>(xs, p);
    } else {
        load_rows<S>(a.seg + (size_t)(tb - t0) * SD, D, d, xs);
    }
    load_cmd(a, tb, d, ubs);
    apply_feedback<MODEL, true>(a, G, hc, ws, xs, tb, off, f_hover, ubs, us, evs);
    fp_ctrl_forward<CTRL>(xs, us, p.fp, p.pid, a.dtc, a.inv_dtc, rc, cs);
}

// ---------------------------------------------------------------------------
// adjoint of one drone's rollout
template <int MODEL, int CTRL, int INTEG, bool AERO, bool EXT, class R>
__device__ __forceinline__ void rollout_bwd_drone(const R& rec, const RollArgs& a, size_t d, int w, int S_h,
                                                  const float* G, float* gl, int gs) {
    constexpr int S = ModelTraits<MODEL, CTRL>::S;
    const size_t D = (size_t)a.D;
    const size_t SD = (size_t)S_h * D;
    DroneParams p;
    load_params<MODEL, CTRL, AERO>(rec, p);
    const float f_hover = (MODEL == MODEL_ID) ? p.id.f_hover : 0.f;
    const RefLane off = ref_lane<EXT>(a, D, d);
    const float seed = a.dloss ? a.dloss[d] : 1.f;
    const float two_seed = 2.f * seed;
    float lam[S];
#pragma unroll
    for (int i = 0; i < S; ++i) lam[i] = 0.f;
    // this drone's gain-gradient contributions, summed in step order, in its own
    // LDS column (registers are the adjoint's scarcest resource): entry k in
    // component k % 4 of the 16-byte quad gq[(k / 4) * gs], so that a step's 52
    // read-modify-writes take 13 quad reads and 13 quad writes (a wave's quads are
    // consecutive: no bank conflicts)
    const bool mlp = EXT && a.mlp_H > 0;
    float4* const gq = reinterpret_cast<float4*>(gl - threadIdx.x) + threadIdx.x;
    if (G && !mlp) {
#pragma unroll
        for (int q = 0; q < NG / 4; ++q) gq[q * gs] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // controller slower than the physics (first-principles, onboard controller):
    // the commands of a block are held over its steps, so their adjoints are
    // summed over the block (rcb) and taken through the controller at its start
    constexpr bool HAS_CTRL = (EXT && MODEL == MODEL_FP && CTRL != CTRL_ROTOR);
    const int n_c = HAS_CTRL ? a.ctrl_every : 1;
    float rch[4] = {0.f, 0.f, 0.f, 0.f}, rcb[4] = {0.f, 0.f, 0.f, 0.f};
    // reward objective: its terms read the neighbouring commands from the command
    // buffer and the attitude of x_{t+1} from memory, so it keeps no values in
    // registers across steps
    const bool rew = EXT && a.has_obj && a.obj_kind == 1;
    const int nseg = (a.T + a.K - 1) / a.K;
    float pn[3];          // position of x_{t+1} of the step being reversed
    // state and command of the next step to reverse, loaded one step ahead so
    // that their memory latency overlaps the current step's arithmetic
    float xq[S], uq[4];
    bool have_q = false, q_ck = false;
    for (int s = nseg - 1; s >= 0; --s) {
        const int t0 = s * a.K;
        const int t1 = min(a.T, t0 + a.K);
        // recompute x_{t0+1} .. x_{t1-1} into segment slots 1..; slot 0 is the
        // checkpoint itself. The state after the segment is the next checkpoint,
        // whose position the previous (later) segment's sweep ended on; the last
        // segment steps once more for the final position.
        const int n_re = (s == nseg - 1) ? (t1 - t0) : (t1 - t0 - 1);
        if (n_re > 0) {
            float x[S], comp[S];
            load_rows<S>(a.ckpt_in + (size_t)s * SD, D, d, x);
            to_dev<MODEL>(x, p);
#pragma unroll
            for (int i = 0; i < S; ++i) comp[i] = 0.f;
            float rcf[4] = {0.f, 0.f, 0.f, 0.f};
            if constexpr (HAS_CTRL) {
                // a segment that starts inside a block (period longer than the
                // checkpoint interval) starts with that block's held commands
                if (t0 % n_c != 0)
                    controller_gains<MODEL, CTRL>(rec, p);
                    block_commands<MODEL, CTRL, S>(a, p, G, gl, gs, off, f_hover, D, d, SD, t0 - t0 % n_c, t0, rcf);
            }
            for (int j = 0; j < n_re; ++j) {
                float u[4], ev[13], ubar[4];
                load_cmd(a, t0 + j, d, ubar);
                apply_feedback<MODEL, EXT>(a, G, gl, gs, x, t0 + j, off, f_hover, ubar, u, ev);
                controller_gains<MODEL, CTRL>(rec, p);
                model_step<MODEL, CTRL, INTEG>(x, comp, u, p, a, rcf, (t0 + j) % n_c == 0);
                if (j + 1 < t1 - t0 || rew) store_rows<S>(a.seg + (size_t)(j + 1) * SD, D, d, x);
            }
            if (s == nseg - 1) {
                pn[0] = x[0]; pn[1] = x[1]; pn[2] = x[2];
            }
        }
        const float* ck = a.ckpt_in + (size_t)s * SD;
        // x_t: the checkpoint itself or a recomputed slot of the segment
        float xc[S], uc[4];
        if (have_q) {
#pragma unroll
            for (int i = 0; i < S; ++i) xc[i] = xq[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) uc[i] = uq[i];
            if (q_ck) to_dev<MODEL>(xc, p);
        } else {
            load_rows<S>((t1 - 1 > t0) ? a.seg + (size_t)(t1 - 1 - t0) * SD : ck, D, d, xc);
            if (!(t1 - 1 > t0)) to_dev<MODEL>(xc, p);
            load_cmd(a, t1 - 1, d, uc);
        }
        for (int t = t1 - 1; t >= t0; --t) {
            // issue the loads of step t - 1: a slot or the checkpoint of this
            // segment, or, with a checkpoint every step, the previous checkpoint
            have_q = false;
            if (t > t0) {
                q_ck = !(t - 1 > t0);
                load_rows<S>(q_ck ? ck : a.seg + (size_t)(t - 1 - t0) * SD, D, d, xq);
                load_cmd(a, t - 1, d, uq);
                have_q = true;
            } else if (a.K == 1 && s > 0) {
                q_ck = true;
                load_rows<S>(a.ckpt_in + (size_t)(s - 1) * SD, D, d, xq);
                load_cmd(a, t - 1, d, uq);
                have_q = true;
            }
            if (a.has_obj) {
                float pr[3];
                ref_pos<EXT>(a, t + 1, off, pr);
                if (rew) {
                    // -exp(-2 |e|) and w_tilt tilt at x_{t+1}: a recomputed slot, the
                    // next checkpoint, or the last segment's final state (extra slot)
                    const float* nx = (t + 1 < t1 || s == nseg - 1) ? a.seg + (size_t)(t + 1 - t0) * SD
                                                                   : a.ckpt_in + (size_t)(s + 1) * SD;
                    float an[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) an[j] = (MODEL == MODEL_FP || j < 2) ? nx[(3 + j) * D + d] : 0.f;
                    const float e0 = pn[0] - pr[0], e1 = pn[1] - pr[1], e2 = pn[2] - pr[2];
                    const float dn = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
                    const float g = dn > 0.f ? seed * 2.f * expf(-2.f * dn) / dn : 0.f;
                    lam[0] += g * e0;
                    lam[1] += g * e1;
                    lam[2] += g * e2;
                    tilt_vjp<MODEL>(an, seed * a.w_tilt, lam);
                } else {
#pragma unroll
                    for (int j = 0; j < 3; ++j) lam[j] += two_seed * (pn[j] - pr[j]);
                }
            }
            float u[4], ev[13];
            apply_feedback<MODEL, EXT>(a, G, gl, gs, xc, t, off, f_hover, uc, u, ev);
            float xb[S];
            float ub[4] = {0.f, 0.f, 0.f, 0.f};
            bool held = false;
            if constexpr (HAS_CTRL) {
                if (n_c > 1) {
                    held = true;
                    const int tb = t - t % n_c;
                    if (t == a.T - 1 || (t + 1) % n_c == 0)   // first visit of this block
                        controller_gains<MODEL, CTRL>(rec, p);
                        block_commands<MODEL, CTRL, S>(a, p, G, gl, gs, off, f_hover, D, d, SD, tb, t0, rch);
                    fp_held_vjp<INTEG>(xc, rch, p.fp, a.dt, a.renorm, lam, xb, rcb);
                    if constexpr (S > S_FP) {
#pragma unroll
                        for (int i = S_FP; i < S; ++i) xb[i] = (t == tb) ? 0.f : lam[i];
                    }
                    if (t == tb) {
                        const float* csb = (S > S_FP) ? lam + S_FP : lam;   // PID state adjoint
                        controller_gains<MODEL, CTRL>(rec, p);
                        fp_ctrl_vjp<CTRL>(xc, u, p.fp, p.pid, a.dtc, a.inv_dtc, rcb, csb, xb, ub);
#pragma unroll
                        for (int i = 0; i < 4; ++i) rcb[i] = 0.f;
                    }
                }
            }
            if (!held) {
                controller_gains<MODEL, CTRL>(rec, p);
                model_step_vjp<MODEL, CTRL, INTEG>(xc, u, p, a, lam, xb, ub);
            }
            if (rew) {
                // action terms: (u_t - u_hover)^2, (u_t - u_{t-1})^2 and, from the
                // next step, (u_{t+1} - u_t)^2
                float ah[4], up[4], un[4];
                hover_action<MODEL, CTRL>(p, ah);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    up[i] = t > 0 ? a.ubuf[((size_t)(t - 1) * 4 + i) * D + d] : ah[i];
                    un[i] = t + 1 < a.T ? a.ubuf[((size_t)(t + 1) * 4 + i) * D + d] : u[i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float gi = a.w_act[i] * (u[i] - ah[i]) + a.w_dact[i] * (u[i] - up[i])
                                     - a.w_dact[i] * (un[i] - u[i]);
                    ub[i] += two_seed * gi;
                }
            } else if (a.has_obj) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ub[i] += two_seed * a.w_u * u[i];
            }
            if (a.g_cmds) {
#pragma unroll
                for (int i = 0; i < 4; ++i) a.g_cmds[((size_t)t * 4 + i) * D + d] = ub[i];
            }
            if (G && mlp) {
                // the policy's activations at e_t (recomputed: a controller block's
                // first visit may have evaluated the policy at another state), its
                // VJP into x_t, and the step's record for the weight gradient
                const MlpView m(G, a.mlp_H);
                const int H = a.mlp_H;
                float o[4], ob[4], eb[13];
                mlp_forward(m, ev, gl, gs, o);
                policy_output_vjp<EXT>(a, o, ub, ob);
#pragma unroll
                for (int j = 0; j < 13; ++j) eb[j] = 0.f;
                mlp_vjp(m, ob, gl, gs, eb);
#pragma unroll
                for (int j = 0; j < 13; ++j) xb[j] += eb[j];
                if (a.mlp_rec) {
                    const size_t TD = (size_t)a.T * D, base = (size_t)t * D + d;
#pragma unroll
                    for (int j = 0; j < 13; ++j) a.mlp_rec[j * TD + base] = ev[j];
                    for (int k = 0; k < H; ++k) {
                        a.mlp_rec[(13 + k) * TD + base] = gl[k * gs];                  // h1
                        a.mlp_rec[(13 + H + k) * TD + base] = gl[(H + k) * gs];        // h2
                        a.mlp_rec[(13 + 2 * H + k) * TD + base] = gl[(3 * H + k) * gs];  // dz1
                        a.mlp_rec[(13 + 3 * H + k) * TD + base] = gl[(2 * H + k) * gs];  // dz2
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) a.mlp_rec[(13 + 4 * H + i) * TD + base] = ob[i];
                }
            } else if (G) {
                float ob[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) ob[i] = ub[i];
                if constexpr (EXT) {
                    if (a.squash) {
                        float o[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float s2 = 0.f;
#pragma unroll
                            for (int j = 0; j < 13; ++j) s2 += G[i * 13 + j] * ev[j];
                            o[i] = s2;
                        }
                        policy_output_vjp<EXT>(a, o, ub, ob);
                    }
                }
#pragma unroll
                for (int j = 0; j < 13; ++j) {
                    float s2 = 0.f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) s2 += G[i * 13 + j] * ob[i];
                    xb[j] += s2;
                }
                float gv[NG];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
#pragma unroll
                    for (int j = 0; j < 13; ++j) gv[i * 13 + j] = ob[i] * ev[j];
                }
#pragma unroll
                for (int q = 0; q < NG / 4; ++q) {
                    float4 s4 = gq[q * gs];
                    s4.x += gv[4 * q];
                    s4.y += gv[4 * q + 1];
                    s4.z += gv[4 * q + 2];
                    s4.w += gv[4 * q + 3];
                    gq[q * gs] = s4;
                }
            }
#pragma unroll
            for (int i = 0; i < S; ++i) lam[i] = xb[i];
            pn[0] = xc[0]; pn[1] = xc[1]; pn[2] = xc[2];
            if (t > t0) {
#pragma unroll
                for (int i = 0; i < S; ++i) xc[i] = xq[i];
#pragma unroll
                for (int i = 0; i < 4; ++i) uc[i] = uq[i];
                if (q_ck) to_dev<MODEL>(xc, p);
            }
        }
    }
    if (a.g_x0) {
        store_rows<S>(a.g_x0, D, d, lam);
        // rows the drone's model does not use (identified drones of a handle with
        // more rows) do not affect the loss
        for (int i = S; i < S_h; ++i) a.g_x0[(size_t)i * D + d] = 0.f;
    }
    if (a.ggc) {
        if (G && !mlp) {
#pragma unroll
            for (int q = 0; q < NG / 4; ++q) {
                const float4 s4 = gq[q * gs];
                a.ggc[(4 * q) * D + d] = s4.x;
                a.ggc[(4 * q + 1) * D + d] = s4.y;
                a.ggc[(4 * q + 2) * D + d] = s4.z;
                a.ggc[(4 * q + 3) * D + d] = s4.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NG; ++i) a.ggc[i * D + d] = 0.f;
        }
    }
}

// The backward reads a checkpoint buffer only while it still holds the tag of
// the forward the host matched; otherwise every requested output of the drone
// is NaN and the handle's device flag is raised (reported as CF_ESTATE).
__device__ __forceinline__ bool ckpt_tag_intact(const RollArgs& a) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 16; ++i) ok &= (a.tag_in[i] == a.tag_exp[i]);
    return ok;
}

__device__ __forceinline__ void poison_gradients(const RollArgs& a, size_t d) {
    const size_t D = (size_t)a.D;
    const float nan = __builtin_nanf("");
    if (a.g_cmds)
        for (size_t i = 0; i < (size_t)a.T * 4; ++i) a.g_cmds[i * D + d] = nan;
    if (a.g_x0)
        for (int i = 0; i < a.S_h; ++i) a.g_x0[(size_t)i * D + d] = nan;
    if (a.ggc)
        for (int i = 0; i < NG; ++i) a.ggc[(size_t)i * D + d] = nan;
    atomicOr(a.dflag, 1u);
}

// ---------------------------------------------------------------------------
// kernels

// A rollout is one long sequential chain per drone, usually with fewer waves
// than SIMDs; when it shares the GPU with wide work (the held step of other
// worlds) its waves take the highest issue priority on their SIMD so the
// chain is not stretched, and the wide work fills the remaining issue slots.
__device__ __forceinline__ void rollout_priority() { __builtin_amdgcn_s_setprio(3); }

template <bool BWD, int MODEL, int CTRL, int INTEG, bool AERO, bool EXT, class R>
__device__ __forceinline__ void rollout_drone(const R& rec, const RollArgs& a, size_t d, int w, int S_h,
                                              const float* G, float* gl, int gs) {
    if constexpr (BWD) {
        rollout_bwd_drone<MODEL, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
    } else {
        rollout_fwd_drone<MODEL, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
    }
}

// EXT: the extended variant, for an onboard controller slower than the physics,
// the BPTT reward objective and the MLP policy; the plain variant keeps the
// registers of the every-step, tracking-loss path with linear feedback
// Dynamic LDS of the rollout kernels: the linear backward keeps each lane's 52
// gain-gradient sums in a column ([52][lanes]); with the MLP policy the
// policies are staged first ([n_pol][P]), followed by each lane's activation
// columns ([2H or 4H][lanes]). Returns the lane's column base.
template <bool EXT>
__device__ __forceinline__ float* stage_policies(const RollArgs& a, float* lds) {
    if constexpr (EXT) {
        if (a.mlp_H > 0) {
            const int n = a.n_pol * a.mlp_P;
            for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = a.gain[i];
            __syncthreads();
            return lds + n + threadIdx.x;
        }
    }
    return lds + threadIdx.x;
}

template <bool BWD, int MODELS, int CTRL, int INTEG, bool AERO, bool EXT>
__global__ __launch_bounds__(256) void k_rollout_lane(RollArgs a, int S_h) {
    rollout_priority();
    extern __shared__ __align__(16) float roll_lds[];
    float* gl = stage_policies<EXT>(a, roll_lds);
    const size_t d = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= (size_t)a.D) return;
    if constexpr (BWD) {
        if (!ckpt_tag_intact(a)) {
            poison_gradients(a, d);
            return;
        }
    }
    const int w = a.drone_world[d];
    const SoaRec rec{a.par_soa, a.M, w};
    const float* G = (a.has_obj && a.gain) ? a.gain + (size_t)a.gidx[w] * NG : nullptr;
    if (EXT && a.mlp_H > 0) G = roll_lds + (size_t)a.gidx[w] * a.mlp_P;
    const int gs = blockDim.x;
    if constexpr (MODELS == MS_FP) rollout_drone<BWD, MODEL_FP, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
    else rollout_drone<BWD, MODEL_ID, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
}

template <bool BWD, int MODELS, int CTRL, int INTEG, bool AERO, bool EXT>
__global__ __launch_bounds__(256) void k_rollout_tile(RollArgs a, const int4* __restrict__ tiles, int S_h) {
    rollout_priority();
    const int4 td = tiles[blockIdx.x];
    const int w = __builtin_amdgcn_readfirstlane(td.x);
    const int d0 = __builtin_amdgcn_readfirstlane(td.y);
    const int cnt = __builtin_amdgcn_readfirstlane(td.z);
    const int model = __builtin_amdgcn_readfirstlane(td.w);
    // the world's feedback gain (or MLP policy), shared by the workgroup, is read from LDS
    __shared__ __align__(16) float sG[NG];
    extern __shared__ __align__(16) float roll_lds[];
    float* gl = stage_policies<EXT>(a, roll_lds);
    const float* G = nullptr;
    if (EXT && a.mlp_H > 0) {
        G = roll_lds + (size_t)a.gidx[w] * a.mlp_P;
    } else if (a.has_obj && a.gain) {
        const float* Gw = a.gain + (size_t)a.gidx[w] * NG;
        for (int i = threadIdx.x; i < NG; i += blockDim.x) sG[i] = Gw[i];
        __syncthreads();
        G = sG;
    }
    if ((int)threadIdx.x >= cnt) return;
    using Rec = typename std::conditional<BWD, ScalarRec, AosRec>::type;
    const Rec rec{a.par_aos + (size_t)w * NREC};
    const size_t d = (size_t)d0 + threadIdx.x;
    if constexpr (BWD) {
        if (!ckpt_tag_intact(a)) {
            poison_gradients(a, d);
            return;
        }
    }
    const int gs = blockDim.x;
    if constexpr (MODELS == MS_FP) {
        rollout_drone<BWD, MODEL_FP, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
    } else if constexpr (MODELS == MS_ID) {
        rollout_drone<BWD, MODEL_ID, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
    } else {
        if (model == MODEL_FP) rollout_drone<BWD, MODEL_FP, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
        else rollout_drone<BWD, MODEL_ID, CTRL, INTEG, AERO, EXT>(rec, a, d, w, S_h, G, gl, gs);
    }
}

template <bool BWD, bool EXT>
static size_t roll_lds_bytes(const RollArgs& a, int lanes) {
    if (EXT && a.mlp_H > 0)
        return ((size_t)a.n_pol * a.mlp_P + (size_t)(BWD ? 4 : 2) * a.mlp_H * lanes) * sizeof(float);
    return BWD ? (size_t)NG * lanes * sizeof(float) : 0;
}

template <bool BWD, int MODELS, int CTRL, int INTEG, bool AERO, bool EXT>
static hipError_t launch_roll_k(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                                hipStream_t s) {
    const int S_h = a.S_h;
    if (ks.mode == LM_LANE) {
        if constexpr (MODELS != MS_BOTH) {
            const int bs = ks.tile;
            const unsigned grid = (unsigned)((a.D + bs - 1) / bs);
            const size_t lds = roll_lds_bytes<BWD, EXT>(a, bs);
            hipLaunchKernelGGL((k_rollout_lane<BWD, MODELS, CTRL, INTEG, AERO, EXT>), dim3(grid), dim3(bs), lds, s,
                               a, S_h);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        const size_t lds = roll_lds_bytes<BWD, EXT>(a, ks.tile);
        hipLaunchKernelGGL((k_rollout_tile<BWD, MODELS, CTRL, INTEG, AERO, EXT>), dim3(n_tiles), dim3(ks.tile), lds,
                           s, a, tiles, S_h);
    }
    return hipGetLastError();
}

// the extended variant serves a slower onboard controller, the reward objective and the MLP policy
template <bool BWD, int MODELS, int CTRL, int INTEG, bool AERO>
static hipError_t launch_roll_t(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                                hipStream_t s) {
    constexpr bool CAN_MR = MODELS != MS_ID && CTRL != CTRL_ROTOR;
    if ((CAN_MR && a.ctrl_every > 1) || (a.has_obj && (a.obj_kind == 1 || a.ref_shift || a.squash)) || a.mlp_H > 0)
        return launch_roll_k<BWD, MODELS, CTRL, INTEG, AERO, true>(ks, a, tiles, n_tiles, s);
    return launch_roll_k<BWD, MODELS, CTRL, INTEG, AERO, false>(ks, a, tiles, n_tiles, s);
}

template <int MODELS, int CTRL, int INTEG, bool AERO>
static hipError_t launch_fwd_t(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                               hipStream_t s) {
    return launch_roll_t<false, MODELS, CTRL, INTEG, AERO>(ks, a, tiles, n_tiles, s);
}
template <int MODELS, int CTRL, int INTEG, bool AERO>
static hipError_t launch_bwd_t(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                               hipStream_t s) {
    return launch_roll_t<true, MODELS, CTRL, INTEG, AERO>(ks, a, tiles, n_tiles, s);
}

#define CF_DISPATCH_A(FN, A, ...)                                                       \
    switch (ks.models * 8 + ks.ctrl * 2 + ks.integ) {                                   \
        case MS_FP * 8 + 0: return FN<MS_FP, CTRL_ROTOR, EULER, A>(__VA_ARGS__);        \
        case MS_FP * 8 + 1: return FN<MS_FP, CTRL_ROTOR, RK4, A>(__VA_ARGS__);          \
        case MS_FP * 8 + 2: return FN<MS_FP, CTRL_PID, EULER, A>(__VA_ARGS__);          \
        case MS_FP * 8 + 3: return FN<MS_FP, CTRL_PID, RK4, A>(__VA_ARGS__);            \
        case MS_FP * 8 + 4: return FN<MS_FP, CTRL_TORQUE, EULER, A>(__VA_ARGS__);       \
        case MS_FP * 8 + 5: return FN<MS_FP, CTRL_TORQUE, RK4, A>(__VA_ARGS__);         \
        case MS_FP * 8 + 6: return FN<MS_FP, CTRL_POSITION, EULER, A>(__VA_ARGS__);     \
        case MS_FP * 8 + 7: return FN<MS_FP, CTRL_POSITION, RK4, A>(__VA_ARGS__);       \
        case MS_ID * 8 + 0: case MS_ID * 8 + 2: case MS_ID * 8 + 4: case MS_ID * 8 + 6: \
            return FN<MS_ID, CTRL_ROTOR, EULER, A>(__VA_ARGS__);                        \
        case MS_ID * 8 + 1: case MS_ID * 8 + 3: case MS_ID * 8 + 5: case MS_ID * 8 + 7: \
            return FN<MS_ID, CTRL_ROTOR, RK4, A>(__VA_ARGS__);                          \
        case MS_BOTH * 8 + 0: return FN<MS_BOTH, CTRL_ROTOR, EULER, A>(__VA_ARGS__);    \
        case MS_BOTH * 8 + 1: return FN<MS_BOTH, CTRL_ROTOR, RK4, A>(__VA_ARGS__);      \
        case MS_BOTH * 8 + 2: return FN<MS_BOTH, CTRL_PID, EULER, A>(__VA_ARGS__);      \
        case MS_BOTH * 8 + 3: return FN<MS_BOTH, CTRL_PID, RK4, A>(__VA_ARGS__);        \
        case MS_BOTH * 8 + 4: return FN<MS_BOTH, CTRL_TORQUE, EULER, A>(__VA_ARGS__);   \
        case MS_BOTH * 8 + 5: return FN<MS_BOTH, CTRL_TORQUE, RK4, A>(__VA_ARGS__);     \
        case MS_BOTH * 8 + 6: return FN<MS_BOTH, CTRL_POSITION, EULER, A>(__VA_ARGS__); \
        case MS_BOTH * 8 + 7: return FN<MS_BOTH, CTRL_POSITION, RK4, A>(__VA_ARGS__);   \
        default: break;                                                                 \
    }
#define CF_DISPATCH(FN, ...)                                                             \
    if (ks.aero) {                                                                       \
        CF_DISPATCH_A(FN, true, __VA_ARGS__)                                             \
    } else {                                                                             \
        CF_DISPATCH_A(FN, false, __VA_ARGS__)                                            \
    }

}  // namespace cfk
