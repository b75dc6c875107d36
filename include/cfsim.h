/*
 * cfsim -- batched drone simulation step for AMD MI355X (gfx950), C interface.
 *
 * The library advances M worlds of N_w drones each (D = sum N_w drones in
 * total) with the two dynamics models of Crazyflow (arXiv 2606.01478,
 * Methods):
 *   - CF_MODEL_FP: first-principles rigid body (Eq. 1) with second-order
 *     thrust / rotor-drag polynomials, the x-airframe mixing matrix and the
 *     adapted, direction-dependent rotor-speed dynamics (Eq. rotor_adapted);
 *     section "First Principles Modeling";
 *   - CF_MODEL_ID: identified attitude-command model (point mass, first-order
 *     collective thrust, second-order attitude response; Eqs. 3_simplified_*);
 *     section "Abstracted Physics Modeling".
 * Control interfaces (section "First Principles Modeling", last paragraphs):
 * rotor speeds, or attitude + collective thrust through a cascaded PID and
 * the motor allocation. Explicit Euler or classical RK4 with the command held
 * over a step (the equations are integrated directly, section "Architecture").
 *
 * Conventions shared by every call
 *   - Memory: every state, command, loss and gradient buffer is caller-owned
 *     device memory, float32, contiguous, structure of arrays: component-major
 *     [component][drone], drones of world 0 first, then world 1, ...
 *     (cf_world_offsets gives the first drone of each world). Buffers passed
 *     to one call must not overlap unless stated.
 *   - Streams: all device work is enqueued on the handle's HIP stream and is
 *     asynchronous; only cf_create, cf_destroy and cf_autotune synchronise.
 *     A handle holding both models owns one more non-blocking stream (its
 *     second per-model launch, forked and joined with events), and a handle
 *     created with CF_F_GRAPH creates a capture stream at its first capture;
 *     no other streams are created.
 *   - Errors: every call returns a cf_status. Argument validation happens on
 *     the host before anything is enqueued; a call that fails validation
 *     writes no output. Asynchronous device faults are reported as
 *     CF_EDEVICE by a later call (sticky) or by cf_last_error.
 *   - Threading: a handle is not thread-safe; distinct handles are
 *     independent.
 */
#ifndef CFSIM_H
#define CFSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cf_status;
#define CF_OK            0
#define CF_EINVAL       (-1)  /* invalid argument (NULL, size, enum, range) */
#define CF_ENODEV       (-2)  /* no usable HIP device */
#define CF_ENOMEM       (-3)  /* device or host allocation failed */
#define CF_EDEVICE      (-4)  /* a HIP runtime call or kernel failed */
#define CF_ESTATE       (-5)  /* call sequence violated (e.g. checkpoint mismatch) */
#define CF_EUNSUPPORTED (-6)  /* valid request that the library does not implement */

/* models, control interfaces, integrators */
#define CF_MODEL_FP      0
#define CF_MODEL_ID      1
#define CF_CTRL_ROTOR    0   /* FP command = rotor-speed setpoints Omega_cmd[4] */
#define CF_CTRL_ATT_PID  1   /* FP command = [roll, pitch, yaw rate, thrust]    */
#define CF_CTRL_TORQUE   2   /* FP command = [thrust, tau_x, tau_y, tau_z] through the
                                motor allocation (CF_P_ALLOC, CF_P_F_MAX)       */
#define CF_CTRL_POSITION 3   /* FP command = [x, y, z, yaw] setpoints through a
                                geometric controller on SO(3) and the allocation:
                                F = m (-kp (p - p_sp) - kv v + g e_z), thrust
                                F . R e_z, desired z axis F/|F| with the commanded
                                yaw, tau = J_ctrl (-kR e_R - kw w) with
                                e_R = vee(R_d^T R - R^T R_d)/2 (CF_P_POS_KP ..
                                CF_P_ATT_KW; no controller state)               */
#define CF_INTEG_EULER   0
#define CF_INTEG_RK4     1

/* cf_desc.flags */
#define CF_F_PLAIN_KERNEL    0x1u  /* cf_step_k: one single-step launch per step   */
#define CF_F_NONFINITE_CHECK 0x2u  /* cf_step_k / cf_rollout: flag non-finite states */
#define CF_F_GRAPH           0x4u  /* replay launch sequences from captured hipGraphs */
#define CF_F_WORKQUEUE       0x8u  /* cf_step_k: persistent work-queue kernel (one launch) */
#define CF_F_NO_AUTOTUNE_CACHE 0x10u /* do not read the autotune cache at create */
#define CF_F_SINGLE_LAUNCH   0x20u  /* mixed-model handles: one launch for both models
                                       (default: one launch per model, forked onto a
                                       second stream and joined with events) */
#define CF_F_TIMING          0x40u  /* cf_step_k: record an event pair around every kernel
                                       launch, or around each graph replay with
                                       CF_F_GRAPH (read with cf_launch_times) */

/*
 * State layout (rows of the [S][D] state):
 *   FP:  0-2 position p [m] (world, z up), 3-6 attitude quaternion (x,y,z,w),
 *        body->world, scalar last; 7-9 velocity v [m/s] (world);
 *        10-12 body rate [rad/s]; 13-16 rotor speeds Omega_1..4.
 *        With CF_CTRL_ATT_PID: 17-18 roll/pitch angle-error integrals,
 *        19-21 body-rate-error integrals, 22-24 body rate of the previous step.
 *   ID:  0-2 p, 3-5 Euler angles (roll, pitch, yaw; R = Rz Ry Rx), 6-8 v,
 *        9-11 Euler-angle rates, 12 collective thrust state f_sum [N].
 * S = 17 (FP rotor, torque or position interface), 25 (FP attitude), 13 (ID). A handle holding both models
 * uses S = max; identified drones use rows 0..12 and leave the rest untouched.
 * Commands are [4][D]: FP rotor: Omega_cmd; FP attitude: [roll, pitch,
 * yaw rate, thrust]; FP torque: [thrust, tau_x, tau_y, tau_z]; FP position:
 * [x, y, z, yaw]; ID: [roll, pitch, yaw, thrust].
 */
#define CF_S_FP_ROTOR 17
#define CF_S_FP_PID   25
#define CF_S_ID       13

/*
 * Per-world parameter record: CF_NPARAM floats, in this order (unused entries
 * must be 0). Units SI. "FP" = read by first-principles worlds, "ID" = by
 * identified worlds, "PID" = by the attitude controller.
 */
#define CF_NPARAM 96
#define CF_P_MASS        0   /* FP,ID  m [kg]                                      */
#define CF_P_GRAVITY     1   /* FP,ID  g [m/s^2], acts along -z                    */
#define CF_P_J           2   /* FP     Jxx, Jyy, Jzz (diagonal inertia) [3]        */
#define CF_P_THRUST      5   /* FP     k0, k1, k2: f_i = k0 + k1 W + k2 W^2 [3]    */
#define CF_P_TORQUE      8   /* FP     t0, t1, t2: drag torque polynomial [3]      */
#define CF_P_MIX_TX     11   /* FP     tau_x = sum mix_tx[i] f_i [4]               */
#define CF_P_MIX_TY     15   /* FP     tau_y = sum mix_ty[i] f_i [4]               */
#define CF_P_MIX_YAW    19   /* FP     tau_z = sum mix_yaw[i] torque_i [4]         */
#define CF_P_MOTOR_UP   23   /* FP     c_v, c_d when Omega_cmd >= Omega [2]        */
#define CF_P_MOTOR_DOWN 25   /* FP     c_v, c_d when Omega_cmd <  Omega [2]        */
#define CF_P_JP         27   /* FP     propeller+motor inertia J_p >= 0 (gyroscopic and
                                      reaction torques; spin directions are -sign(mix_yaw)) */
#define CF_P_DRAG       28   /* FP,ID  linear body-frame drag C_a diagonal [3]: the force is
                                      R C_a R^T v (entries <= 0 damp)               */
#define CF_P_ANG_KP     31   /* PID    roll/pitch angle P gain [1/s] [2]           */
#define CF_P_ANG_KI     33   /* PID    roll/pitch angle I gain [1/s^2] [2]         */
#define CF_P_RATE_KP    35   /* PID    body-rate P gain [1/s] [3]                  */
#define CF_P_RATE_KI    38   /* PID    body-rate I gain [1/s^2] [3]                */
#define CF_P_RATE_KD    41   /* PID    body-rate D gain [-] [3]                    */
#define CF_P_J_CTRL     44   /* PID    inertia used by the controller [3]          */
#define CF_P_F_MAX      47   /* PID    per-rotor thrust limit [N]                  */
#define CF_P_ALLOC      48   /* PID    4x4 row-major: f = alloc [T, tau_x, tau_y, tau_z] */
#define CF_P_CF         64   /* ID     thrust scaling c_f                          */
#define CF_P_CTAU       65   /* ID     thrust time coefficient c_tau [1/s], >= 0;
                                0 selects the variant without thrust dynamics: the
                                commanded thrust acts directly and state row 12 holds
                                the applied thrust (12 dynamic states)            */
#define CF_P_CPSI1      66   /* ID     attitude coefficient c1 per axis [3]        */
#define CF_P_CPSI2      69   /* ID     c2 per axis [3]                             */
#define CF_P_CPSI3      72   /* ID     c3 per axis [3]                             */
#define CF_P_POS_KP     75   /* POS    position gain per axis [1/s^2] [3]          */
#define CF_P_POS_KV     78   /* POS    velocity gain per axis [1/s] [3]            */
#define CF_P_ATT_KR     81   /* POS    attitude-error gain per axis [1/s^2] [3]    */
#define CF_P_ATT_KW     84   /* POS    body-rate gain per axis [1/s] [3]           */

typedef struct cf_desc {
    int32_t n_worlds;                 /* M >= 1                                       */
    int32_t n_drones;                 /* drones per world when drones_per_world NULL  */
    const int32_t* drones_per_world;  /* host [M], each >= 0, or NULL                 */
    int32_t model;                    /* CF_MODEL_* of every world when model_per_world NULL */
    const uint8_t* model_per_world;   /* host [M] or NULL                             */
    int32_t control;                  /* CF_CTRL_* for first-principles worlds        */
    int32_t integrator;               /* CF_INTEG_*                                   */
    float dt;                         /* step [s], finite, > 0                        */
    int32_t renorm_q;                 /* 1: normalise the quaternion after each step  */
    const float* params;              /* host [M][CF_NPARAM]; copied at create        */
    int32_t n_gains;                  /* feedback gains available to cf_rollout (>= 0) */
    const int32_t* gain_index;        /* host [M] in [0, n_gains) or NULL (all 0)     */
    void* stream;                     /* hipStream_t, NULL = default stream           */
    uint32_t flags;                   /* CF_F_*                                       */
    int32_t device;                   /* HIP device ordinal, -1 = current device      */
    int32_t ctrl_every;               /* onboard controller every n physics steps (0, 1: every step) */
} cf_desc;

/*
 * Control rate (the paper runs its controllers at 50-500 Hz on a faster
 * physics loop; section "Architecture", control interfaces). With
 * ctrl_every = n > 1 the onboard controller of first-principles worlds
 * (attitude PID, position controller, torque allocation) is evaluated at the
 * start of every block of n physics steps with period n dt (the PID's
 * integrators and derivative use it) and its rotor-speed commands are held,
 * zero-order, over the block; the PID state rows change only at evaluations.
 * The rotor interface and identified worlds have no onboard controller and
 * ignore it. Blocks are counted from the first step of each cf_step_k call
 * (k must be a multiple of n) and from t = 0 in cf_rollout (T need not be;
 * ckpt_every K must divide n or be a multiple of it). The plain single-step
 * kernel (CF_F_PLAIN_KERNEL) launches once per block. n <= CF_MAX_CTRL_EVERY.
 */
#define CF_MAX_CTRL_EVERY 4096

typedef struct cf_handle cf_handle;

/*
 * Tracking objective and linear feedback of cf_rollout / cf_rollout_backward.
 * Applied command u_t = ubar_t + G_w (x_t[0:13] - x_ref(t)) when gain != NULL
 * (with policy_hidden > 0 the small-MLP policy's output replaces G_w (...);
 * with policy_scale set, that output o enters as policy_scale * tanh(o)).
 * Loss per drone: sum_{t=1..T} |p_t - p_ref(t)|^2 + w_u sum_{t=0..T-1} |u_t|^2,
 * t_n = (ref_step0 + n) dt (+ s_d with ref_time_shift). Reference (ref_table == NULL): figure-eight
 * p_ref = [A sin(2 pi t/P), (A/2) sin(4 pi t/P), 0] + offset_d and its
 * derivative; x_ref = [p_ref, (0,0,0,1), v_ref, 0] (FP) or
 * [p_ref, 0, v_ref, 0, m g / c_f] (ID). With ref_table, x_ref(t) is row t
 * (offset added to its position).
 */
typedef struct cf_objective {
    const float* gain;        /* device [n_gains][4][13] or NULL (no feedback)   */
    const float* ref_table;   /* device [T+1][13] or NULL (figure-eight)         */
    float ref_amp;            /* A [m]                                           */
    float ref_period;         /* P [s], > 0                                      */
    const float* ref_offset;  /* device [3][D] or NULL                           */
    float w_u;                /* command weight, >= 0                            */
    int32_t kind;             /* CF_OBJ_TRACKING (0) or CF_OBJ_BPTT_REWARD (1)   */
    float w_tilt;             /* reward: tilt weight, >= 0                       */
    float w_act[4];           /* reward: weights of (u - u_hover)^2, >= 0        */
    float w_dact[4];          /* reward: weights of (u_t - u_{t-1})^2, >= 0      */
    int32_t policy_hidden;    /* 0: linear feedback, gain [n_gains][4][13]; H in
                                 1..CF_MLP_MAX_HIDDEN: small-MLP policies in gain,
                                 [n_gains][CF_MLP_PARAMS(H)] (see below)          */
    int32_t ref_step0;        /* figure-eight: step n of the rollout tracks the
                                 reference at t = (ref_step0 + n) dt, >= 0, so that
                                 consecutive rollouts continue along it          */
    const float* ref_time_shift; /* device [D] or NULL; figure-eight only: drone d
                                 tracks the reference at t_n + s_d, which places
                                 starts along the trajectory (Methods,
                                 "Backpropagation Through Time"). The phase
                                 2 pi s_d / P is formed in binary32: keep |s_d|
                                 within a few periods. Selects the extended
                                 kernel variant.                                 */
    float policy_scale[4];    /* all 0: the policy output o is added to ubar as
                                 is. Else u_i = ubar_i + policy_scale[i] tanh(o_i),
                                 each >= 0: actions normalised to [-1, 1] that map
                                 linearly onto command ranges, as the paper states
                                 for its policies' action space (Methods, "Proximal
                                 Policy Optimization"); selects the extended kernel
                                 variant.                                        */
} cf_objective;

/*
 * Small-MLP policy (the actor network of the paper's BPTT setup, Methods,
 * "Backpropagation Through Time"; its architecture is not printed, this is
 * the library's): u_t = ubar_t + W3 tanh(W2 tanh(W1 e_t + b1) + b2) + b3 with
 * e_t = x_t[0:13] - x_ref(t), H units per hidden layer. Each policy is packed
 * [W1 (H x 13, row-major) | b1 (H) | W2 (H x H) | b2 (H) | W3 (4 x H) | b3 (4)],
 * CF_MLP_PARAMS(H) = 13 H + H + H H + H + 4 H + 4 floats; world w uses policy
 * gain_index[w]. The backward's g_gain receives the gradient in the same packing.
 * Limits: (n_gains * CF_MLP_PARAMS(H) + 4 * 64 * H) * 4 bytes <= 64 KiB (the
 * policies and each lane's activations live in LDS), and the handle's tile
 * size must be 64 lanes when its worlds are tiled (CF_EUNSUPPORTED otherwise).
 * The backward keeps (17 + 4 H) floats per drone-step of scratch for the
 * weight-gradient reduction.
 */
#define CF_MLP_MAX_HIDDEN 32
#define CF_MLP_PARAMS(H) (13 * (H) + (H) + (H) * (H) + (H) + 4 * (H) + 4)

/*
 * Objective kinds. CF_OBJ_TRACKING: the loss above. CF_OBJ_BPTT_REWARD: minus
 * the summed reward of the paper's BPTT tracking task (Methods,
 * "Backpropagation Through Time"), for t = 0..T-1 with u_t the applied command
 * and x_{t+1} the state it leads to:
 *   r_t = exp(-2 |p_{t+1} - p_ref(t+1)|) - w_tilt tilt(x_{t+1})
 *         - sum_i w_act_i (u_t,i - u_hover,i)^2 - sum_i w_dact_i (u_t,i - u_{t-1},i)^2,
 * tilt = angle between the body and world z axes, u_{-1} = u_hover, the hover
 * command of the drone's interface (identified [0, 0, 0, m g / c_f]; attitude
 * [0, 0, 0, m g]; torque [m g, 0, 0, 0]; rotor: the reference speed on every
 * rotor). Norms take gradient 0 at their kinks. Not for the position interface
 * (CF_EINVAL). w_u is unused. The forward keeps the applied commands in the
 * checkpoint buffer for the backward.
 */
#define CF_OBJ_TRACKING    0
#define CF_OBJ_BPTT_REWARD 1

/*
 * cf_create (the simulation data of Methods, "Architecture": one structure
 * holding every buffer of a batch of parallel worlds x drones per world x data,
 * Fig. 1; parameters and state as stated in "First Principles Modeling" and
 * "Abstracted Physics Modeling"): validate *desc, copy the parameter records
 * and the world layout to the device, choose kernel variants (autotune cache
 * unless CF_F_NO_AUTOTUNE_CACHE) and return a handle in *out (NULL on failure).
 * The handle owns its device copies; desc and the arrays it points to may be
 * freed by the caller after the call.
 * Errors: CF_EINVAL (NULL pointers, M < 1, negative drone counts, D > 2^31-1,
 * unknown enum, dt not finite or <= 0, a non-finite parameter, mass/inertia/
 * k2/c_f not > 0, J_p < 0, c_tau < 0, gain index out of range), CF_ENODEV (no device),
 * CF_ENOMEM, CF_EDEVICE.
 */
cf_status cf_create(const cf_desc* desc, cf_handle** out);

/* cf_destroy: synchronise the stream and free everything the library owns (the
   counterpart of cf_create). NULL is a no-op. */
cf_status cf_destroy(cf_handle* h);

/* Queries (host only) of the batch layout (worlds x drones x data, Methods,
   "Architecture"): rows S of the state, total drones D, and the first drone of
   each world, offsets_host[M + 1] (host memory, written by the call). Errors:
   CF_EINVAL for NULL arguments. cf_set_stream replaces the handle's stream
   (a hipStream_t, NULL = default stream); later calls enqueue on it. */
cf_status cf_state_dim(const cf_handle* h, int32_t* S);
cf_status cf_total_drones(const cf_handle* h, int64_t* D);
cf_status cf_world_offsets(const cf_handle* h, int64_t* offsets_host /* [M+1] */);
cf_status cf_set_stream(cf_handle* h, void* stream);

/*
 * cf_reset (continuous/masked resets, Methods, "Architecture", last paragraph): for every world w
 * with world_mask[w] != 0 (all worlds when world_mask is NULL), copy the S rows
 * of init into state for that world's drones. state, init: device [S][D];
 * world_mask: device uint8 [M] or NULL. state and init must not overlap.
 * Errors: CF_EINVAL (NULL handle, buffers not device memory of S*D floats,
 * overlapping buffers, mask smaller than M bytes), sticky CF_EDEVICE.
 */
cf_status cf_reset(cf_handle* h, float* state, const float* init, const uint8_t* world_mask);

/*
 * cf_step_k (the simulation step of Methods, "Architecture": the equations of
 * motion of "First Principles Modeling" / "Abstracted Physics Modeling"
 * integrated directly, successive steps fused like the paper's scan over
 * steps; control interfaces of "First Principles Modeling", last paragraph):
 * advance every drone k >= 1 steps with the command held (zero-order
 * hold). state: device [S][D], updated in place; cmd: device [4][D].
 * nonfinite_world: device uint32 [M] or NULL; with CF_F_NONFINITE_CHECK the
 * entry of a world is OR-ed with 1 when any of its drones ends with a
 * non-finite state component (the buffer is not cleared by the library).
 * Kernel: fused k-step kernel that keeps the state in registers (chunked by
 * the autotuned K), or k single-step launches with CF_F_PLAIN_KERNEL, or the
 * persistent work-queue kernel (CF_F_WORKQUEUE or autotune choice).
 * With a controller period of n > 1 steps (cf_desc.ctrl_every), k must be a
 * multiple of n (CF_EINVAL otherwise). Errors: CF_EINVAL (k < 1, buffers not
 * device memory of the stated sizes), sticky CF_EDEVICE.
 */
cf_status cf_step_k(cf_handle* h, float* state, const float* cmd, int32_t k,
                    uint32_t* nonfinite_world);

/*
 * Checkpoint buffer of cf_rollout / cf_rollout_backward (device, caller-owned,
 * cf_ckpt_floats floats): the states at t = 0, K, 2K, ... as [ceil(T/K)][S][D];
 * for the reward objective then the applied commands u_t as [T][4][D] (its
 * backward needs their neighbours); then CF_CKPT_TAG_FLOATS 32-bit words that
 * tag the forward that filled it (handle, a per-handle generation count, T, K,
 * S, D, objective kind and a hash of the objective's weights and of which of
 * its optional inputs are present).
 */
#define CF_CKPT_TAG_FLOATS 16

/* cf_ckpt_floats: floats of the checkpoint buffer for (T, K, objective kind) on
   this handle, in *n (host). Errors: CF_EINVAL (NULL, T < 1, K < 1, unknown kind). */
cf_status cf_ckpt_floats(const cf_handle* h, int32_t T, int32_t ckpt_every, int32_t kind, int64_t* n);

/*
 * cf_rollout (Results, "Computation Performance", and Methods,
 * "Backpropagation Through Time": rollouts whose objective is differentiated
 * through the simulation steps): T >= 1 steps from x0 (device [S][D]) with
 * per-step commands cmds (device [T][4][D], the ubar_t of cf_objective). obj
 * may be NULL (no feedback, no loss: loss and loss_world must then be NULL).
 * ckpt_every K >= 1; ckpt (device, cf_ckpt_floats(h, T, K, kind) floats, or
 * NULL) receives the checkpoint states, the reward objective's applied
 * commands and the tag; it is required by cf_rollout_backward.
 * x_T (device [S][D]), traj (device [T+1][S][D]), loss (device [D]) and
 * loss_world (device [M], per-world sums in a fixed order) may each be NULL.
 * Errors: CF_EINVAL (T < 1, K < 1, K neither a divisor nor a multiple of the
 * controller period, loss without obj, a buffer smaller than stated, an
 * objective field out of range), sticky CF_EDEVICE.
 */
cf_status cf_rollout(cf_handle* h, const float* x0, const float* cmds, int32_t T,
                     const cf_objective* obj, int32_t ckpt_every, float* ckpt,
                     float* x_T, float* traj, float* loss, float* loss_world);

/*
 * cf_rollout_backward (Results, "Computation Performance": gradients of an
 * objective with respect to the control inputs through the simulation steps
 * and the onboard controllers; Methods, "Architecture": differentiability of
 * the whole pipeline): gradient of sum_d dloss[d] * loss_d (dloss: device [D],
 * NULL = ones) through the whole rollout, by a hand-written discrete adjoint
 * that recomputes each K-step segment from its checkpoint. cmds, T, obj and
 * ckpt_every must be those of the cf_rollout that filled ckpt on this handle
 * (x0 is not read: the checkpoint holds it). Checked on the host against the
 * tags of this handle's forwards: a buffer that no forward of this handle
 * filled, or filled with another T, K or objective, returns CF_ESTATE and
 * writes nothing. Checked again on the device against the tag in the buffer:
 * a buffer overwritten since (by another handle's forward, or reused memory)
 * makes the kernel write NaN to every requested output and sets the handle's
 * sticky status to CF_ESTATE, reported by cf_last_error. Any number of
 * forwards may precede their backwards. Outputs (overwritten, each may be
 * NULL): g_cmds device [T][4][D] (d/d ubar_t), g_x0 device [S][D], g_gain
 * device [n_gains][4][13] (sum over drones in a fixed order; requires
 * obj->gain). Errors: CF_EINVAL (sizes as in cf_rollout, NULL ckpt, g_gain
 * without a gain), CF_ESTATE, sticky CF_EDEVICE.
 */
cf_status cf_rollout_backward(cf_handle* h, const float* x0, const float* cmds, int32_t T,
                              const cf_objective* obj, int32_t ckpt_every, const float* ckpt,
                              const float* dloss, float* g_cmds, float* g_x0, float* g_gain);

/*
 * cf_rollout_backward_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving or training loops, harnesses
 * that forbid hipMalloc). The same gradients as cf_rollout_backward, with the
 * same arguments, ownership and errors, but every scratch buffer (the
 * figure-eight table, recomputed segment states, per-drone gain-gradient terms
 * and the gain reduction's partial sums) lives in one static device array of
 * CF_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from the first
 * cf_create on that GPU until the process ends; the call allocates nothing.
 * A request whose scratch exceeds the array returns CF_EINVAL before any work:
 * it needs (T + 1) * 6 floats with a figure-eight objective, plus
 * (min(K, T) + 1{reward}) * S * D floats when that is more than one state, plus
 * 52 * D + n_gains * 52 * min(1024, ceil(D / 2048)) floats with g_gain, each
 * rounded up to 64 floats. Every call on one GPU uses the same array, so calls
 * that overlap on one GPU (other streams, other handles, other threads) race;
 * nothing in it needs to start at zero.
 */
#define CF_NOALLOC_SCRATCH_BYTES (64u << 20)
cf_status cf_rollout_backward_noalloc(cf_handle* h, const float* x0, const float* cmds, int32_t T,
                                      const cf_objective* obj, int32_t ckpt_every, const float* ckpt,
                                      const float* dloss, float* g_cmds, float* g_x0, float* g_gain);

/*
 * cf_autotune (the paper leaves kernel fusion and scheduling to its JIT
 * compiler, Methods, "Architecture"; here the launch shape is chosen by
 * measurement): time candidate launch shapes of cf_step_k (fused grid vs
 * persistent work queue, tile size, steps per launch K) on copies of state and
 * cmd (device [S][D], [4][D], not modified) for about budget_ms, keep the
 * fastest for this handle and store it in the autotune cache file
 * ($CFSIM_AUTOTUNE_CACHE, default $HOME/.cache/cfsim_autotune.txt: one line per
 * handle signature with the chosen shape and its time; the signature is the
 * device architecture, worlds, drones, first-principles worlds, interface,
 * integrator, whether drag or rotor inertia is present, and the control
 * interval). Synchronises.
 */
cf_status cf_autotune(cf_handle* h, const float* state, const float* cmd, int32_t k, int32_t budget_ms);

/* cf_launch_config: current launch choice (host, written by the call): use_workqueue (bit 0: work queue; bit 1: one launch per
   model on two streams), tile (lanes per work item), chunk K (0 = all k steps per launch). */
cf_status cf_launch_config(const cf_handle* h, int32_t* use_workqueue, int32_t* tile, int32_t* chunk);

/* cf_set_launch_config: pin the launch choice of cf_step_k (the values
   cf_launch_config reports): use_wq bit 0 work queue, bit 1 one launch per model
   on two streams (mixed handles); tile 64, 128 or 256 lanes; chunk steps per
   launch (0 = all k steps in one launch; a multiple of the controller period);
   wq_waves: with the work queue, at most this many of its waves resident per
   compute unit (0 = as many as fit; 1..128; a compute unit has four SIMDs),
   which leaves registers and issue slots to kernels on other streams. Replaces
   the autotuned choice until the next cf_autotune (which resets wq_waves to 0).
   Errors: CF_EINVAL. */
cf_status cf_set_launch_config(cf_handle* h, int32_t use_wq, int32_t tile, int32_t chunk, int32_t wq_waves);

/* cf_launch_times (measurement of the kernels against their rooflines): with
   CF_F_TIMING, the durations in ms of the kernel launches of the latest
   cf_step_k call on stream slot 0 (the
   handle's stream: every launch of a single-model or single-launch handle, the
   first-principles launches of a mixed handle) or slot 1 (the identified-model
   launches of a mixed handle), from HIP events recorded on that stream around
   each launch. A handle with CF_F_GRAPH times each replay as a whole instead:
   one entry on slot 0 (events around the graph launch), none on slot 1.
   ms: host [max_n], the first min(max_n, *n) entries are written;
   *n: the number of timed launches (at most 512 per slot and call). Waits for
   those events. Errors: CF_EINVAL (NULL, slot not 0 or 1, no CF_F_TIMING),
   CF_EDEVICE. */
cf_status cf_launch_times(cf_handle* h, int32_t slot, float* ms, int32_t max_n, int32_t* n);

/* cf_strerror: static text of a status (never NULL). */
const char* cf_strerror(cf_status status);

/* cf_last_error: synchronise the stream and return the sticky status (CF_OK,
   CF_EDEVICE after a device fault, CF_ESTATE after a backward found its
   checkpoint buffer overwritten). */
cf_status cf_last_error(cf_handle* h);

/* ---- sampled-rollout controller ---------------------------------------------
 * The iCEM/MPPI hybrid of the obstacle-avoidance showcase (Methods, section
 * "Model Predictive Path Integral"; Results, MPPI paragraph): C independent
 * controllers, each samples N command sequences of H steps around its previous
 * mean with temporally correlated noise, rolls every sample through the
 * simulator from the current state, keeps its n_e lowest-cost samples (the
 * paper keeps the best 1 %) and replaces its mean by their exponentially
 * weighted average; the controller with the lowest elite cost supplies the
 * command. Per sample k of controller c at call `iteration`:
 *   xi_t    standard normals: Philox4x64-10 with counter (t/2, k, c, iteration)
 *           and key (seed, 0); each 64-bit output word w gives one Box-Muller
 *           pair from u1 = ((lo32(w) >> 9) + 1/2) 2^-23, u2 = ((hi32(w) >> 9) +
 *           1/2) 2^-23; words 0..3 give components 0..3 of step 2b and then of
 *           step 2b+1 (in the order cos, sin of each pair);
 *   eps_0 = xi_0, eps_t = beta eps_{t-1} + sqrt(1 - beta^2) xi_t; eps = 0 for k = 0;
 *   u_t = clip(mean[c][min(t + shift, H - 1)] + sigma * eps_t, u_lo, u_hi);
 *   x advanced `substeps` simulator steps per u_t (the handle's model,
 *   interface, integrator and dt); cost
 *   J = sum_t sum_i r_u[i] (u_t,i - u_ref[i])^2 + sum_{t=1..H} q_p |p_t - goal|^2
 *       + q_v |v_t|^2 + w_obs sum_o max(0, 1 - |p_t - c_o|^2 / r_o^2)^2,
 *   a non-finite J counted as +inf.
 * Elites: the n_e smallest (J, k) pairs; new mean = sum w_k u_k / sum w_k with
 * w_k = exp(-(J_k - J_min) / lambda). best = argmin_c J_min,c (lowest c on ties),
 * u_apply = new mean[best][0].
 */
#define CF_MPPI_MAX_OBSTACLES 16
#define CF_MPPI_MAX_ELITE 4096

typedef struct cf_mppi cf_mppi;

typedef struct cf_mppi_desc {
    int32_t n_controllers;   /* 1 <= C <= 65535                                       */
    int32_t n_samples;       /* N >= 1 per controller, C*N <= 2^31-1                  */
    int32_t horizon;         /* H >= 1                                                */
    int32_t substeps;        /* simulator steps per horizon step, >= 1               */
    int32_t n_elite;         /* 1 <= n_e <= min(N, CF_MPPI_MAX_ELITE)                 */
    float sigma[4];          /* noise scale per command component, >= 0               */
    float beta;              /* temporal correlation, 0 <= beta < 1                   */
    float lambda;            /* temperature of the elite weights, > 0                 */
    float u_lo[4], u_hi[4];  /* command bounds, u_lo <= u_hi                          */
    float u_ref[4], r_u[4];  /* command cost: reference and weight (>= 0)             */
    float goal[3];           /* position goal [m]                                     */
    float q_p, q_v, w_obs;   /* position, velocity and obstacle weights, >= 0         */
    int32_t n_obstacles;     /* 0 .. CF_MPPI_MAX_OBSTACLES                            */
    float obstacles[CF_MPPI_MAX_OBSTACLES][4];  /* centre [m], radius [m] (> 0)       */
    uint64_t seed;           /* generator key                                         */
} cf_mppi_desc;

/*
 * cf_mppi_create: a controller set for the single world of handle h (h must
 * have n_worlds = 1; its parameters, model, interface, integrator and dt are
 * used; h must outlive the controller set and its stream is used). Allocates
 * device scratch of about C*N*4 + C*n_e*(16*H + 8) bytes.
 * Errors: CF_EINVAL (h has more than one world, a field out of range or not
 * finite), CF_ENOMEM; *out is NULL on failure.
 */
cf_status cf_mppi_create(cf_handle* h, const cf_mppi_desc* desc, cf_mppi** out);

/* cf_mppi_destroy: synchronise the stream and free the scratch. NULL is a no-op. */
cf_status cf_mppi_destroy(cf_mppi* m);

/*
 * cf_mppi_step: one control step of all controllers, asynchronous on the
 * handle's stream. x_now device [S] (the handle's state layout); mean device
 * [C][H][4], in: the previous plans (read shifted by `shift` >= 0 steps), out:
 * the new plans. Optional device outputs (NULL to skip): u_apply [4], best [1],
 * cost [C][N], elite_idx [C][n_e] (ordered by cost, then index), cost_min [C].
 * The same (seed, iteration) gives the same samples. Calls on one controller
 * set share its scratch and must not overlap on different streams.
 * Errors: CF_EINVAL (NULL or too-small device buffers, shift < 0), sticky
 * CF_EDEVICE.
 */
cf_status cf_mppi_step(cf_mppi* m, const float* x_now, float* mean, int32_t shift, uint64_t iteration,
                       float* u_apply, int32_t* best, float* cost, int32_t* elite_idx, float* cost_min);

/* cf_mppi_noise: the correlated noise eps (before sigma and clipping) of call
   `iteration`, device [C][N][H][4]; zero for sample 0. */
cf_status cf_mppi_noise(cf_mppi* m, uint64_t iteration, float* eps);

/* ---- measurement helper ----------------------------------------------------
 * cf_probe_fma: launch n_blocks workgroups of 256 lanes, each lane running 8
 * independent FP32 FMA chains of `iters` steps (16 * iters FLOP per lane), on
 * `stream` (hipStream_t, NULL = default), writing one float per lane to the
 * device buffer out [n_blocks * 256]. form 0: a <- a b + c with b = 0.9999999,
 * c = 1e-7 (three-operand FMA); form 1: a <- b c + a with b = 1e-3, c = 1e-4
 * (two-operand accumulate form). Timing it gives the achievable unpacked FP32
 * FMA rate that the simulation kernels' VALU roofline is compared with.
 * Errors: CF_EINVAL (NULL or too-small out, n_blocks < 1, iters < 1, form not
 * 0 or 1), CF_EDEVICE.
 */
cf_status cf_probe_fma(float* out, int32_t n_blocks, int32_t iters, int32_t form, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CFSIM_H */
