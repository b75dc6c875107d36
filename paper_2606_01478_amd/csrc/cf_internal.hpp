// Internal interface between the host runtime and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfk {

// bit set of models present in a launch
enum : int { MS_FP = 1, MS_ID = 2, MS_BOTH = 3 };
// how lanes are mapped to drones
//   LM_LANE: lane = drone, world looked up per lane, parameters from the
//            transposed [NREC][M] copy (worlds of a handful of drones);
//   LM_TILE: one workgroup per tile. Rollouts take per-world tiles {world,
//            first drone, count, model} (parameters are uniform loads); held
//            steps take packed tiles {first list entry, count, model} of one
//            model that may span worlds (a wave within one world reads its
//            parameters with uniform loads, a wave across worlds per lane);
//   LM_WQ:   persistent workgroups pop packed tiles from an atomic queue head.
enum : int { LM_LANE = 0, LM_TILE = 1, LM_WQ = 2 };

struct KernelSel {
    int models;  // MS_*
    int ctrl;    // CTRL_ROTOR / CTRL_PID
    int integ;   // EULER / RK4
    int mode;    // LM_*
    int tile;    // lanes per workgroup (64, 128, 256)
    int aero;    // kernels with gyroscopic/reaction torques, drag and the general rotor law compiled in
};

struct StepArgs {
    float* st;              // [S][D]
    const float* cmd;       // [4][D]
    int64_t D;
    int M;
    const float* par_aos;   // [M][NREC]
    const float* par_soa;   // [NREC][M]
    const int32_t* drone_world;  // [D]
    float dt;
    float dtc, inv_dtc;     // onboard controller period (ctrl_every physics steps) and its inverse
    int ctrl_every;         // the controller runs on every ctrl_every-th step (launches start on one)
    int renorm;
    int K;                  // steps per launch
    uint32_t* nonfinite;    // [M] or null
    const int32_t* plist;   // [D] drones in packed-tile order (tile kernels)
};

struct RollArgs {
    const float* x0;        // [S][D]
    int S_h;                // rows of the handle's state (stride between checkpoints)
    const float* cmds;      // [T][4][D]
    int T;
    int64_t D;
    int M;
    const float* par_aos;
    const float* par_soa;
    const int32_t* drone_world;
    float dt;
    float dtc, inv_dtc;     // onboard controller period and its inverse
    int ctrl_every;         // the controller runs on steps t with t % ctrl_every == 0
    int renorm;
    // objective
    int has_obj;
    const float* gain;      // [G][4][13] or null
    const int32_t* gidx;    // [M] device
    const float* ref_tab;   // [T+1][6] figure-eight (p, v) or [T+1][13] user table
    int ref_user;
    const float* ref_off;   // [3][D] or null
    const float* ref_shift; // [D] per-drone reference time shift [s] or null (extended kernels)
    float ref_w, ref_inv_w; // figure-eight angular rate 2 pi / P and its inverse
    float w_u;
    int obj_kind;           // 0: tracking loss, 1: BPTT reward
    float w_tilt, w_act[4], w_dact[4];
    float* ubuf;            // reward: applied commands [T][4][D] inside the checkpoint buffer
                            // (written by the forward, read by the backward) or null
    int mlp_H;              // small-MLP policy width (0: linear feedback through `gain`)
    int squash;             // policy output o enters as act_s * tanh(o) (extended kernels)
    float act_s[4];
    int mlp_P;              // floats per policy
    int n_pol;              // policies in `gain` (staged into LDS)
    float* mlp_rec;         // backward: per drone-step records [17 + 4 H][T][D] for the
                            // weight-gradient reduction
    // forward outputs
    int K;                  // checkpoint interval
    float* ckpt;            // [ceil(T/K)][S][D] or null
    float* xT;
    float* traj;            // [T+1][S][D] or null
    float* loss;            // [D] or null
    uint32_t* nonfinite;
    // backward
    const float* ckpt_in;
    const uint32_t* tag_in;  // the tag words at the end of ckpt_in
    uint32_t tag_exp[16];    // the tag the host matched for this buffer
    uint32_t* dflag;         // set to 1 when tag_in differs from tag_exp
    const float* dloss;     // [D] or null (ones)
    float* g_cmds;          // [T][4][D] or null
    float* g_x0;            // [S][D] or null
    float* ggc;             // [52][D] per-drone gain-gradient contributions or null
    float* seg;             // [K][S][D] segment scratch
};

// sampled-rollout controller (one world's model, C controllers x N samples)
constexpr int MPPI_MAX_OBS = 16;
constexpr int MPPI_MAX_ELITE = 4096;
constexpr int MPPI_SELECT_THREADS = 1024;
struct MppiArgs {
    const float* par;        // the world's record [NREC]
    const float* x_now;      // [S]
    const float* mean;       // [C][H][4] previous plan (read at min(t + shift, H - 1))
    float* mean_out;         // [C][H][4] new plan (may alias mean)
    int C, N, H, sub, n_e, shift;
    float dt;
    float dtc, inv_dtc;      // onboard controller period and its inverse
    int ctrl_every;          // controller on physics steps t * sub + s divisible by it
    int renorm;
    float sigma[4], beta, beta_c, inv_lambda;
    float u_lo[4], u_hi[4], u_ref[4], r_u[4];
    float goal[3], q_p, q_v, w_obs;
    int n_obs;
    float obs[MPPI_MAX_OBS][4];  // centre, 1 / r^2
    uint64_t seed, iter;
    float* cost;             // [C][N]
    float* eps_out;          // [C][N][H][4] (noise kernel only)
    float* elite_u;          // scratch [C][H*4][n_e]
    int32_t* elite_idx;      // [C][n_e]
    float* elite_cost;       // [C][n_e]
    float* cost_min;         // [C]
    float* u_apply;          // [4] or null
    int32_t* best;           // [1] or null
};
hipError_t launch_mppi_rollout(const KernelSel& ks, const MppiArgs& a, hipStream_t s);
hipError_t launch_mppi_noise(const MppiArgs& a, hipStream_t s);
hipError_t launch_mppi_select(const MppiArgs& a, hipStream_t s);

hipError_t launch_step(const KernelSel& ks, const StepArgs& a, const int4* tiles, int n_tiles,
                       unsigned* counter, int wq_blocks, hipStream_t s);
hipError_t launch_rollout_fwd(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                              hipStream_t s);
hipError_t launch_rollout_bwd(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                              hipStream_t s);
// resident workgroups per CU of the work-queue kernel for this selection
int step_wq_blocks_per_cu(const KernelSel& ks);

}  // namespace cfk
