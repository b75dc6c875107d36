// Held-command step kernels: K steps per launch with each drone's state in
// registers (K = 1 is the plain single-step kernel), in three lane mappings
// (per-lane world, one world per tile, persistent work queue over tiles).
#include "cf_device.hpp"
#include "cf_internal.hpp"

namespace cfk {

// One drone, K steps with a held command; state rows st[i*D + d].
// MR: variant for an onboard controller slower than the physics
template <int MODEL, int CTRL, int INTEG, bool AERO, bool MR, class R>
__device__ __forceinline__ void run_held(const R& rec, const StepArgs& a, size_t d, int w) {
    const size_t D = (size_t)a.D;
    bool bad = false;
    if constexpr (MODEL == MODEL_FP) {
        constexpr int S = (CTRL == CTRL_PID) ? S_PID : S_FP;
        const FpParams P = load_fp<AERO>(rec);
        float x[S], u[4], comp[S_FP];
#pragma unroll
        for (int i = 0; i < S; ++i) x[i] = a.st[i * D + d];
        rotors_to_dev(x, P);
#pragma unroll
        for (int i = 0; i < S_FP; ++i) comp[i] = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) u[i] = a.cmd[i * D + d];
        float rc[4] = {0.f, 0.f, 0.f, 0.f};   // held rotor commands
        int phase = 0;                        // launches start on a controller step
        for (int k = 0; k < a.K; ++k) {
            const bool ctrl_now = MR ? phase == 0 : true;
            // the controller's gains are read where it runs (scalar loads of the
            // world's record) rather than held in registers through the integration
            PidParams C;
            if constexpr (CTRL != CTRL_ROTOR) {
                if (ctrl_now) C = load_pid(laundered(rec), CTRL == CTRL_POSITION);
            }
            fp_step<CTRL, INTEG>(x, comp, u, P, C, a.dt, a.dtc, a.inv_dtc, a.renorm, rc, ctrl_now);
            if constexpr (MR) {
                if (++phase == a.ctrl_every) phase = 0;
            }
        }
        rotors_from_dev(x, P);
        // the row addresses are formed again here rather than kept from the loads
        // through the step loop (where they would take registers or scratch)
        size_t ds = d;
        asm volatile("" : "+v"(ds));
#pragma unroll
        for (int i = 0; i < S; ++i) {
            a.st[i * D + ds] = x[i];
            bad |= !isfinite(x[i]);
        }
    } else {
        const IdParams P = load_id<AERO>(rec);
        float x[S_ID], u[4], comp[S_ID];
#pragma unroll
        for (int i = 0; i < S_ID; ++i) { x[i] = a.st[i * D + d]; comp[i] = 0.f; }
#pragma unroll
        for (int i = 0; i < 4; ++i) u[i] = a.cmd[i * D + d];
        // the start angles' sines and cosines: exact every 8th step, in between
        // carried from the previous step by the angle addition
        EulerBase B;
        for (int k = 0; k < a.K; ++k) {
            if ((k & 7) == 0) euler_base(x + 3, B);
            else euler_rebase(x + 3, B);
            id_step_base<INTEG>(x, comp, u, P, a.dt, B);
        }
        size_t ds = d;
        asm volatile("" : "+v"(ds));
#pragma unroll
        for (int i = 0; i < S_ID; ++i) {
            a.st[i * D + ds] = x[i];
            bad |= !isfinite(x[i]);
        }
    }
    if (a.nonfinite && bad) atomicOr(a.nonfinite + w, 1u);
}

template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR, class R>
__device__ __forceinline__ void run_model(int model, const R& rec, const StepArgs& a, size_t d, int w) {
    if constexpr (MODELS == MS_FP) {
        run_held<MODEL_FP, CTRL, INTEG, AERO, MR>(rec, a, d, w);
    } else if constexpr (MODELS == MS_ID) {
        run_held<MODEL_ID, CTRL, INTEG, AERO, MR>(rec, a, d, w);
    } else {
        if (model == MODEL_FP) run_held<MODEL_FP, CTRL, INTEG, AERO, MR>(rec, a, d, w);
        else run_held<MODEL_ID, CTRL, INTEG, AERO, MR>(rec, a, d, w);
    }
}

// A packed tile: `count` consecutive entries of the drone list from `first`, all
// of one model, possibly of several worlds (every tile but each model's last is
// full, so no lanes idle at world ends). A wave whose lanes share one world
// reads that world's parameters with scalar loads into scalar registers; a wave
// across a world boundary reads each lane's own with vector loads.
template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR>
__device__ __forceinline__ void run_tile(const StepArgs& a, int4 td) {
    // td = {first list entry, drone count, model, 0}, uniform over the workgroup
    const int first = __builtin_amdgcn_readfirstlane(td.x);
    const int cnt = __builtin_amdgcn_readfirstlane(td.y);
    const int model = __builtin_amdgcn_readfirstlane(td.z);
    const int lane = threadIdx.x;
    if (lane >= cnt) return;
    const size_t d = (size_t)a.plist[first + lane];
    const int w = a.drone_world[d];
    const int w0 = __builtin_amdgcn_readfirstlane(w);
    if (__builtin_amdgcn_ballot_w64(w != w0) == 0) {
        run_model<MODELS, CTRL, INTEG, AERO, MR>(model, AosRec{a.par_aos + (size_t)w0 * NREC}, a, d, w0);
    } else {
        run_model<MODELS, CTRL, INTEG, AERO, MR>(model, LaneRec{a.par_aos + (size_t)w * NREC}, a, d, w);
    }
}

template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR>
__global__ __launch_bounds__(256) void k_step_lane(StepArgs a) {
    const size_t d = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= (size_t)a.D) return;
    const int w = a.drone_world[d];
    const SoaRec rec{a.par_soa, a.M, w};
    if constexpr (MODELS == MS_FP) run_held<MODEL_FP, CTRL, INTEG, AERO, MR>(rec, a, d, w);
    else run_held<MODEL_ID, CTRL, INTEG, AERO, MR>(rec, a, d, w);
}

template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR>
__global__ __launch_bounds__(256) void k_step_tile(StepArgs a, const int4* __restrict__ tiles) {
    run_tile<MODELS, CTRL, INTEG, AERO, MR>(a, tiles[blockIdx.x]);
}

// Persistent work queue: each workgroup pops the next tile index from *counter
// until the tiles run out; every workgroup exits after one failed pop.
template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR>
__device__ __forceinline__ void run_queue(const StepArgs& a, const int4* __restrict__ tiles, int n_tiles,
                                          unsigned* counter) {
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (t >= n_tiles) break;
        run_tile<MODELS, CTRL, INTEG, AERO, MR>(a, tiles[t]);
    }
}

template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR>
__global__ __launch_bounds__(256) void k_step_wq(StepArgs a, const int4* __restrict__ tiles, int n_tiles,
                                                 unsigned* counter) {
    run_queue<MODELS, CTRL, INTEG, AERO, MR>(a, tiles, n_tiles, counter);
}



template <int MODELS, int CTRL, int INTEG, bool AERO, bool MR>
static hipError_t launch_step_k(const KernelSel& ks, const StepArgs& a, const int4* tiles, int n_tiles,
                                unsigned* counter, int wq_blocks, hipStream_t s) {
    if (ks.mode == LM_LANE) {
        if constexpr (MODELS == MS_BOTH) return hipErrorInvalidValue;
        const int bs = ks.tile;
        const unsigned grid = (unsigned)((a.D + bs - 1) / bs);
        hipLaunchKernelGGL((k_step_lane<MODELS, CTRL, INTEG, AERO, MR>), dim3(grid), dim3(bs), 0, s, a);
    } else if (ks.mode == LM_TILE) {
        hipLaunchKernelGGL((k_step_tile<MODELS, CTRL, INTEG, AERO, MR>), dim3(n_tiles), dim3(ks.tile), 0, s, a, tiles);
    } else {
        // work-queue workgroups that do not fit at once start later, find the
        // queue empty and exit
        hipLaunchKernelGGL((k_step_wq<MODELS, CTRL, INTEG, AERO, MR>), dim3(wq_blocks), dim3(ks.tile), 0, s, a, tiles,
                           n_tiles, counter);
    }
    return hipGetLastError();
}

// the slow-controller variant exists only where there is an onboard controller
template <int MODELS, int CTRL, int INTEG, bool AERO>
static hipError_t launch_step_t(const KernelSel& ks, const StepArgs& a, const int4* tiles, int n_tiles,
                                unsigned* counter, int wq_blocks, hipStream_t s) {
    if constexpr (MODELS != MS_ID && CTRL != CTRL_ROTOR) {
        if (a.ctrl_every > 1)
            return launch_step_k<MODELS, CTRL, INTEG, AERO, true>(ks, a, tiles, n_tiles, counter, wq_blocks, s);
    }
    return launch_step_k<MODELS, CTRL, INTEG, AERO, false>(ks, a, tiles, n_tiles, counter, wq_blocks, s);
}

template <int MODELS, int CTRL, int INTEG, bool AERO>
static int wq_blocks_t(int tile) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_wq<MODELS, CTRL, INTEG, AERO, false>, tile, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
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

hipError_t launch_step(const KernelSel& ks, const StepArgs& a, const int4* tiles, int n_tiles,
                       unsigned* counter, int wq_blocks, hipStream_t s) {
    CF_DISPATCH(launch_step_t, ks, a, tiles, n_tiles, counter, wq_blocks, s)
    return hipErrorInvalidValue;
}

int step_wq_blocks_per_cu(const KernelSel& ks) {
    CF_DISPATCH(wq_blocks_t, ks.tile)
    return 1;
}

}  // namespace cfk
