// Sampled-rollout controller (the iCEM / MPPI hybrid of the paper's obstacle
// avoidance showcase): every lane is one sample of one controller. It draws its
// temporally correlated command noise from a counter-based generator on the
// fly (nothing is stored), rolls the sample through the model and writes only
// its cost. A workgroup per controller then selects the elites by radix select
// over (cost, sample index), regenerates the elites' commands from their
// counters and forms the exponentially weighted mean in a fixed order.
#include "cf_device.hpp"
#include "cf_internal.hpp"

namespace cfk {

// ---- Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------------------------
constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ull, PH_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ull, PH_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        const uint64_t hi0 = __umul64hi((unsigned long long)PH_M0, (unsigned long long)x[0]), lo0 = PH_M0 * x[0];
        const uint64_t hi1 = __umul64hi((unsigned long long)PH_M1, (unsigned long long)x[2]), lo1 = PH_M1 * x[2];
        const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
    }
}

// open-interval uniform from the top 23 bits, exact in binary32
__device__ __forceinline__ float unit_open(uint32_t u) { return ((float)(u >> 9) + 0.5f) * 0x1p-23f; }

// eight standard normals of block b of sample (k, c) at iteration `iter`:
// each 64-bit word gives one Box-Muller pair from its (low, high) halves;
// the hardware sine and cosine take their argument in revolutions, so
// sin(2 pi u2) is one instruction with no range reduction (u2 in (0, 1))
__device__ __forceinline__ void normals8(uint64_t b, uint64_t k, uint64_t c, const MppiArgs& a, float z[8]) {
    uint64_t x[4] = {b, k, c, a.iter};
    philox4x64(x, a.seed, 0ull);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const float u1 = unit_open((uint32_t)x[w]);
        const float u2 = unit_open((uint32_t)(x[w] >> 32));
        const float r = sqrt_hw(-2.f * logf(u1));
        z[2 * w] = r * __builtin_amdgcn_cosf(u2);
        z[2 * w + 1] = r * __builtin_amdgcn_sinf(u2);
    }
}

// Sequential generator of one sample's correlated noise eps_t (t = 0, 1, ...):
// first-order autoregressive filter with unit stationary variance; sample 0
// is the noise-free mean.
struct NoiseSeq {
    uint64_t k, c;
    float eps[4], z[8];
    float scale;  // 0 for sample 0
    __device__ __forceinline__ void init(uint64_t k_, uint64_t c_) {
        k = k_;
        c = c_;
        scale = k_ == 0 ? 0.f : 1.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) eps[i] = 0.f;
    }
    // advance to step t (called with t = 0, 1, 2, ... in order); even steps draw
    // a new block, odd steps use its second half (selected, not indexed, so z
    // stays in registers)
    __device__ __forceinline__ void next(int t, const MppiArgs& a) {
        if ((t & 1) == 0) normals8((uint64_t)(t >> 1), k, c, a, z);
        const bool odd = (t & 1) != 0;
        float zi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) zi[i] = odd ? z[4 + i] : z[i];
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) eps[i] = zi[i];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) eps[i] = a.beta * eps[i] + a.beta_c * zi[i];
        }
    }
    // sampled command at step t: clip(mean + sigma eps)
    __device__ __forceinline__ void command(int t, const MppiArgs& a, float u[4]) const {
        const int ts = min(t + a.shift, a.H - 1);
        const float* m = a.mean + ((size_t)c * a.H + ts) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) u[i] = fminf(fmaxf(m[i] + a.sigma[i] * (scale * eps[i]), a.u_lo[i]), a.u_hi[i]);
    }
};

// ---- rollout + cost: one lane per sample ---------------------------------------
// MR: variant for an onboard controller slower than the physics
template <int MODEL, int CTRL, int INTEG, bool AERO, bool MR>
__global__ __launch_bounds__(256) void k_mppi_rollout(MppiArgs a) {
    const int c = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.N) return;
    const VecRec rec(a.par);
    constexpr int S = MODEL == MODEL_ID ? S_ID : (CTRL == CTRL_PID ? S_PID : S_FP);
    constexpr int V = MODEL == MODEL_ID ? 6 : 7;  // first velocity row
    float x[S], comp[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        x[i] = a.x_now[i];
        comp[i] = 0.f;
    }
    FpParams P;
    PidParams Cp;
    IdParams Pi;
    if constexpr (MODEL == MODEL_FP) {
        P = load_fp<AERO>(rec);
        if constexpr (CTRL != CTRL_ROTOR) Cp = load_pid(rec, CTRL == CTRL_POSITION);
        rotors_to_dev(x, P);
    } else {
        Pi = load_id<AERO>(rec);
    }
    NoiseSeq ns;
    ns.init((uint64_t)k, (uint64_t)c);
    float J = 0.f;
    float rc[4] = {0.f, 0.f, 0.f, 0.f};   // held rotor commands
    int phase = 0;                        // physics step within the controller period
    for (int t = 0; t < a.H; ++t) {
        ns.next(t, a);
        float u[4];
        ns.command(t, a, u);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float du = u[i] - a.u_ref[i];
            J += a.r_u[i] * du * du;
        }
        for (int s = 0; s < a.sub; ++s) {
            if constexpr (MODEL == MODEL_FP) {
                fp_step<CTRL, INTEG>(x, comp, u, P, Cp, a.dt, a.dtc, a.inv_dtc, a.renorm, rc, MR ? phase == 0 : true);
                if constexpr (MR) {
                    if (++phase == a.ctrl_every) phase = 0;
                }
            } else {
                id_step<INTEG>(x, comp, u, Pi, a.dt);
            }
        }
        const float ex = x[0] - a.goal[0], ey = x[1] - a.goal[1], ez = x[2] - a.goal[2];
        J += a.q_p * (ex * ex + ey * ey + ez * ez) +
             a.q_v * (x[V] * x[V] + x[V + 1] * x[V + 1] + x[V + 2] * x[V + 2]);
        for (int o = 0; o < a.n_obs; ++o) {
            const float dx = x[0] - a.obs[o][0], dy = x[1] - a.obs[o][1], dz = x[2] - a.obs[o][2];
            const float pen = fmaxf(1.f - (dx * dx + dy * dy + dz * dz) * a.obs[o][3], 0.f);
            J += a.w_obs * pen * pen;
        }
    }
    a.cost[(size_t)c * a.N + k] = isfinite(J) ? J : __builtin_inff();
}

// correlated noise only (eps, before sigma and clipping), [C][N][H][4]
__global__ __launch_bounds__(256) void k_mppi_noise(MppiArgs a) {
    const int c = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.N) return;
    NoiseSeq ns;
    ns.init((uint64_t)k, (uint64_t)c);
    float* out = a.eps_out + ((size_t)c * a.N + k) * a.H * 4;
    for (int t = 0; t < a.H; ++t) {
        ns.next(t, a);
#pragma unroll
        for (int i = 0; i < 4; ++i) out[t * 4 + i] = ns.scale * ns.eps[i];
    }
}

// ---- elite selection and weighted mean: one workgroup per controller ------------
// order-preserving map of a binary32 to an unsigned key
__device__ __forceinline__ uint32_t ordered_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(MPPI_SELECT_THREADS) void k_mppi_select(MppiArgs a) {
    constexpr int BS = MPPI_SELECT_THREADS;
    __shared__ unsigned hist[256];
    __shared__ uint64_t keys[MPPI_MAX_ELITE];
    __shared__ float wts[MPPI_MAX_ELITE];
    __shared__ uint64_t s_prefix, s_mask;
    __shared__ int s_need, s_eq, s_count;
    __shared__ float s_wsum;
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const float* J = a.cost + (size_t)c * a.N;
    // visit every sample's key; loads are issued UNR at a time so their
    // latencies overlap (one workgroup per controller has few waves to hide them)
    constexpr int UNR = 8;
    auto for_each_key = [&](auto&& fn) {
        for (int64_t k0 = tid; k0 < a.N; k0 += BS * UNR) {
            float v[UNR];
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const int64_t k = k0 + j * BS;
                v[j] = k < a.N ? J[k] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const int64_t k = k0 + j * BS;
                if (k < a.N) fn(((uint64_t)ordered_bits(v[j]) << 32) | (uint32_t)k);
            }
        }
    };

    // ascending bitonic sort of keys[0, P2), P2 a power of two (all threads)
    auto bitonic = [&](int P2) {
        for (int size = 2; size <= P2; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = tid; i < P2 / 2; i += BS) {
                    const int lo = 2 * i - (i & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t x = keys[lo], y = keys[hi];
                    if ((x > y) == up) {
                        keys[lo] = y;
                        keys[hi] = x;
                    }
                }
                __syncthreads();
            }
        }
    };

    // Common case: a threshold key just above the n_e-th smallest, taken from a
    // sorted sample of the keys; one pass collects every key at or below it
    // (one LDS atomic per wave) and the candidates are sorted. The radix select
    // below is the fallback when the candidates are too few or too many.
    bool selected = false;
    if (2 * a.n_e <= MPPI_MAX_ELITE) {
        constexpr int SAMPLE = 2048;
        const int ns = (int)(a.N < SAMPLE ? a.N : SAMPLE);
        int P2s = 1;
        while (P2s < ns) P2s <<= 1;
        for (int i = tid; i < P2s; i += BS) {
            uint64_t key = ~0ull;
            if (i < ns) {
                const int64_t k = (int64_t)i * a.N / ns;
                key = ((uint64_t)ordered_bits(J[k]) << 32) | (uint32_t)k;
            }
            keys[i] = key;
        }
        __syncthreads();
        bitonic(P2s);
        int r = (ns == a.N) ? a.n_e - 1
                            : (int)ceilf((float)ns * (float)a.n_e / (float)a.N * 1.25f) + 8;
        r = r < ns - 1 ? r : ns - 1;
        const uint64_t tau = keys[r];
        if (tid == 0) s_count = 0;
        __syncthreads();   // tau read everywhere before keys[] is reused
        for (int64_t k0 = 0; k0 < a.N; k0 += (int64_t)BS * UNR) {
            float v[UNR];
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const int64_t k = k0 + j * BS + tid;
                v[j] = k < a.N ? J[k] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const int64_t k = k0 + j * BS + tid;
                const uint64_t key = ((uint64_t)ordered_bits(v[j]) << 32) | (uint32_t)k;
                const bool f = (k < a.N) && key <= tau;
                const uint64_t m = __ballot(f);
                const int nw = __popcll(m);
                int base = 0;
                if (lane == 0 && nw) base = atomicAdd(&s_count, nw);
                base = __shfl(base, 0, 64);
                const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
                if (f && pos < MPPI_MAX_ELITE) keys[pos] = key;
            }
        }
        __syncthreads();
        const int cnt = s_count;
        if (cnt >= a.n_e && cnt <= MPPI_MAX_ELITE) {
            int P2 = 1;
            while (P2 < cnt) P2 <<= 1;
            for (int i = cnt + tid; i < P2; i += BS) keys[i] = ~0ull;
            __syncthreads();
            bitonic(P2);
            selected = true;
        }
        __syncthreads();
    }
    if (!selected) {
        // radix select of the n_e-th smallest key, 8 bits per pass from the top;
        // stops once every key left in the chosen bucket is taken
        if (tid == 0) {
            s_prefix = 0;
            s_mask = 0;
            s_need = a.n_e;
        }
        __syncthreads();
        for (int pass = 0; pass < 8; ++pass) {
            const int sh = 56 - 8 * pass;
            if (tid < 256) hist[tid] = 0;
            __syncthreads();
            const uint64_t prefix = s_prefix, mask = s_mask;
            for_each_key([&](uint64_t key) {
                if ((key & mask) == prefix) atomicAdd(&hist[(key >> sh) & 255u], 1u);
            });
            __syncthreads();
            if (wave == 0) {
                const int need = s_need;
                const unsigned h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                               h3 = hist[4 * lane + 3];
                const unsigned tot = h0 + h1 + h2 + h3;
                unsigned incl = tot;
    #pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const unsigned v = __shfl_up(incl, off, 64);
                    if (lane >= off) incl += v;
                }
                const unsigned excl = incl - tot;
                const bool here = excl < (unsigned)need && (unsigned)need <= incl;
                if (here) {
                    unsigned cum = excl;
                    const unsigned hh[4] = {h0, h1, h2, h3};
                    int dig = 0;
    #pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (cum + hh[j] >= (unsigned)need) {
                            dig = 4 * lane + j;
                            s_need = need - (int)cum;
                            s_eq = (int)hh[j];
                            break;
                        }
                        cum += hh[j];
                    }
                    s_prefix = prefix | ((uint64_t)dig << sh);
                    s_mask = mask | (255ull << sh);
                }
            }
            __syncthreads();
            if (s_eq == s_need) break;
        }
        // collect the n_e keys with (key & mask) <= prefix, then sort them
        const uint64_t prefix = s_prefix, mask = s_mask;
        int P2 = 1;
        while (P2 < a.n_e) P2 <<= 1;
        for (int i = tid; i < P2; i += BS) keys[i] = ~0ull;
        if (tid == 0) s_count = 0;
        __syncthreads();
        for_each_key([&](uint64_t key) {
            if ((key & mask) <= prefix) {
                const int pos = atomicAdd(&s_count, 1);
                if (pos < a.n_e) keys[pos] = key;
            }
        });
        __syncthreads();
        bitonic(P2);
    }
    // weights exp(-(J - J_min) / lambda)
    const float jmin = from_ordered((uint32_t)(keys[0] >> 32));
    for (int i = tid; i < a.n_e; i += BS) {
        const float ji = from_ordered((uint32_t)(keys[i] >> 32));
        wts[i] = expf(-(ji - jmin) * a.inv_lambda);
        a.elite_idx[(size_t)c * a.n_e + i] = (int32_t)(uint32_t)keys[i];
        a.elite_cost[(size_t)c * a.n_e + i] = ji;
    }
    // regenerate each elite's commands into [H*4][n_e]
    float* eu = a.elite_u + (size_t)c * a.H * 4 * a.n_e;
    for (int i = tid; i < a.n_e; i += BS) {
        NoiseSeq ns;
        ns.init((uint64_t)(uint32_t)keys[i], (uint64_t)c);
        for (int t = 0; t < a.H; ++t) {
            ns.next(t, a);
            float u[4];
            ns.command(t, a, u);
#pragma unroll
            for (int j = 0; j < 4; ++j) eu[(size_t)(t * 4 + j) * a.n_e + i] = u[j];
        }
    }
    __syncthreads();
    // fixed-order sums: lanes stride over elites, butterfly within the wave
    if (wave == 0) {
        float s = 0.f;
        for (int i = lane; i < a.n_e; i += 64) s += wts[i];
        s = wave_sum(s);
        if (lane == 0) s_wsum = s;
    }
    __syncthreads();
    const float inv_w = 1.f / s_wsum;
    for (int j = wave; j < a.H * 4; j += BS / 64) {
        const float* row = eu + (size_t)j * a.n_e;
        float s = 0.f;
        for (int i = lane; i < a.n_e; i += 64) s += wts[i] * row[i];
        s = wave_sum(s);
        if (lane == 0) a.mean_out[(size_t)c * a.H * 4 + j] = s * inv_w;
    }
    if (tid == 0) a.cost_min[c] = jmin;
}

// controller with the lowest elite cost (ties to the lower index) and its first command
__global__ void k_mppi_pick(MppiArgs a) {
    if (threadIdx.x != 0) return;
    int b = 0;
    for (int c = 1; c < a.C; ++c)
        if (a.cost_min[c] < a.cost_min[b]) b = c;
    if (a.best) a.best[0] = b;
    if (a.u_apply)
        for (int j = 0; j < 4; ++j) a.u_apply[j] = a.mean_out[(size_t)b * a.H * 4 + j];
}

template <int MODEL, int CTRL, int INTEG, bool AERO>
static hipError_t launch_roll(const KernelSel&, const MppiArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.N + 255) / 256), (unsigned)a.C);
    if constexpr (MODEL == MODEL_FP && CTRL != CTRL_ROTOR) {
        if (a.ctrl_every > 1) {
            hipLaunchKernelGGL((k_mppi_rollout<MODEL, CTRL, INTEG, AERO, true>), grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_mppi_rollout<MODEL, CTRL, INTEG, AERO, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

#define CF_MPPI_DISPATCH_A(A)                                                                \
    switch (ks.models * 8 + ks.ctrl * 2 + ks.integ) {                                        \
        case MS_FP * 8 + 0: return launch_roll<MODEL_FP, CTRL_ROTOR, EULER, A>(ks, a, s);    \
        case MS_FP * 8 + 1: return launch_roll<MODEL_FP, CTRL_ROTOR, RK4, A>(ks, a, s);      \
        case MS_FP * 8 + 2: return launch_roll<MODEL_FP, CTRL_PID, EULER, A>(ks, a, s);      \
        case MS_FP * 8 + 3: return launch_roll<MODEL_FP, CTRL_PID, RK4, A>(ks, a, s);        \
        case MS_FP * 8 + 4: return launch_roll<MODEL_FP, CTRL_TORQUE, EULER, A>(ks, a, s);   \
        case MS_FP * 8 + 5: return launch_roll<MODEL_FP, CTRL_TORQUE, RK4, A>(ks, a, s);     \
        case MS_FP * 8 + 6: return launch_roll<MODEL_FP, CTRL_POSITION, EULER, A>(ks, a, s); \
        case MS_FP * 8 + 7: return launch_roll<MODEL_FP, CTRL_POSITION, RK4, A>(ks, a, s);   \
        case MS_ID * 8 + 0: case MS_ID * 8 + 2: case MS_ID * 8 + 4: case MS_ID * 8 + 6:      \
            return launch_roll<MODEL_ID, CTRL_ROTOR, EULER, A>(ks, a, s);                    \
        case MS_ID * 8 + 1: case MS_ID * 8 + 3: case MS_ID * 8 + 5: case MS_ID * 8 + 7:      \
            return launch_roll<MODEL_ID, CTRL_ROTOR, RK4, A>(ks, a, s);                      \
        default: break;                                                                      \
    }

hipError_t launch_mppi_rollout(const KernelSel& ks, const MppiArgs& a, hipStream_t s) {
    if (ks.aero) {
        CF_MPPI_DISPATCH_A(true)
    } else {
        CF_MPPI_DISPATCH_A(false)
    }
    return hipErrorInvalidValue;
}

hipError_t launch_mppi_noise(const MppiArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.N + 255) / 256), (unsigned)a.C);
    hipLaunchKernelGGL(k_mppi_noise, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mppi_select(const MppiArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_mppi_select, dim3((unsigned)a.C), dim3(MPPI_SELECT_THREADS), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mppi_pick, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace cfk
