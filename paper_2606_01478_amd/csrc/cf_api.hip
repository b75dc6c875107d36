// Host runtime of the C interface declared in include/cfsim.h: argument
// validation, device-side world layout, tile lists for uneven worlds, launch
// selection, hipGraph replay of launch sequences, the autotuner, and the small
// utility kernels (reset, reference table, deterministic reductions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cfsim.h"
#include "cf_device.hpp"
#include "cf_host.hpp"
#include "cf_internal.hpp"

using namespace cfk;

// ---------------------------------------------------------------------------
// utility kernels

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

struct TagWords {
    uint32_t w[CF_CKPT_TAG_FLOATS];
};

// the forward's tag at the end of its checkpoint buffer
__global__ void k_write_tag(uint32_t* dst, TagWords t) {
    const int i = threadIdx.x;
    if (i < CF_CKPT_TAG_FLOATS) dst[i] = t.w[i];
}

// state[:, d] = init[:, d] for drones of masked worlds
__global__ void k_reset(float* __restrict__ st, const float* __restrict__ init, int S, int64_t D,
                        const int32_t* __restrict__ drone_world, const uint8_t* __restrict__ mask) {
    const size_t d = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= (size_t)D) return;
    if (mask && !mask[drone_world[d]]) return;
    for (int i = 0; i < S; ++i) st[(size_t)i * D + d] = init[(size_t)i * D + d];
}

// figure-eight (lemniscate of Gerono) rows [p(3), v(3)] for steps t = 0..T of a
// rollout that starts at reference step step0
__global__ void k_eight_table(float* tab, int T, float dt, float amp, float period, int step0) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T) return;
    const double w0 = 2.0 * 3.14159265358979323846 / (double)period;
    const double tt = ((double)step0 + (double)t) * (double)dt;
    const double A = amp;
    float* r = tab + (size_t)t * 6;
    r[0] = (float)(A * sin(w0 * tt));
    r[1] = (float)(0.5 * A * sin(2.0 * w0 * tt));
    r[2] = 0.f;
    r[3] = (float)(A * w0 * cos(w0 * tt));
    r[4] = (float)(A * w0 * cos(2.0 * w0 * tt));
    r[5] = 0.f;
}

// out[w][c] = sum over the drones of world w of v[c][d], in a fixed order:
// each thread sums a strided subset, then a fixed LDS tree.
__global__ __launch_bounds__(256) void k_reduce_world(const float* __restrict__ v, int ncomp, int64_t D,
                                                      const int64_t* __restrict__ off, float* __restrict__ out) {
    __shared__ float sh[256];
    const int w = blockIdx.x;
    const int64_t a = off[w], b = off[w + 1];
    for (int c = 0; c < ncomp; ++c) {
        float s = 0.f;
        for (int64_t d = a + threadIdx.x; d < b; d += blockDim.x) s += v[(size_t)c * D + d];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[(size_t)w * ncomp + c] = sh[0];
        __syncthreads();
    }
}

// Gain gradient g[k][c] = sum over drones d whose world uses gain k of
// v[c][d] (c < 52), in a fixed order that depends only on D and the grid:
// stage 1, workgroup b of gain k sums the drones of chunk b (each thread a
// strided subset, then an LDS tree per component) into part[k][b][c];
// stage 2 sums part[k][0..nb) in order. O(D / (nb 256) + log 256 + nb) deep.
constexpr int GAIN_COMP = 52;
constexpr int GAIN_MAX_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_gain_partial(const float* __restrict__ v, int64_t D,
                                                      const int32_t* __restrict__ drone_world,
                                                      const int32_t* __restrict__ gidx, int64_t chunk,
                                                      float* __restrict__ part) {
    __shared__ float sh[256];
    const int b = blockIdx.x, k = blockIdx.y, nb = gridDim.x;
    const int64_t lo = (int64_t)b * chunk, hi = min(D, lo + chunk);
    float acc[GAIN_COMP];
#pragma unroll
    for (int c = 0; c < GAIN_COMP; ++c) acc[c] = 0.f;
    for (int64_t d = lo + threadIdx.x; d < hi; d += blockDim.x) {
        if (gidx[drone_world[d]] != k) continue;
#pragma unroll
        for (int c = 0; c < GAIN_COMP; ++c) acc[c] += v[(size_t)c * D + d];
    }
    for (int c = 0; c < GAIN_COMP; ++c) {
        sh[threadIdx.x] = acc[c];
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[((size_t)k * nb + b) * GAIN_COMP + c] = sh[0];
        __syncthreads();
    }
}

__global__ void k_gain_final(const float* __restrict__ part, int nb, float* __restrict__ g) {
    const int k = blockIdx.x, c = threadIdx.x;
    if (c >= GAIN_COMP) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[((size_t)k * nb + b) * GAIN_COMP + c];
    g[(size_t)k * GAIN_COMP + c] = s;
}

// Weight gradient of the small-MLP policies from the reverse sweep's records
// rec[r][n] (n = t D + d; rows: e 13, h1 H, h2 H, dz1 H, dz2 H, d3 4):
//   dW1 = sum_n dz1 e^T, db1 = sum_n dz1, dW2 = sum_n dz2 h1^T, db2 = sum_n dz2,
//   dW3 = sum_n d3 h2^T, db3 = sum_n d3,
// over the drones whose world uses policy k, in the packing of the policy. Stage 1:
// workgroup b of policy k stages tiles of 64 records into LDS (zero for other
// policies' drones) and each thread accumulates its parameters over the tiles of
// chunk b; stage 2 sums the chunks in order.
constexpr int MLP_MAX_P = 2048;   // CF_MLP_PARAMS(CF_MLP_MAX_HIDDEN) = 1636
constexpr int MLP_PER_THREAD = MLP_MAX_P / 256;

__device__ __forceinline__ void mlp_param_rows(int p, int H, int* ra, int* rb) {
    const int E = 0, H1 = 13, H2 = 13 + H, DZ1 = 13 + 2 * H, DZ2 = 13 + 3 * H, D3 = 13 + 4 * H;
    if (p < 13 * H) { *ra = DZ1 + p / 13; *rb = E + p % 13; return; }
    p -= 13 * H;
    if (p < H) { *ra = DZ1 + p; *rb = -1; return; }
    p -= H;
    if (p < H * H) { *ra = DZ2 + p / H; *rb = H1 + p % H; return; }
    p -= H * H;
    if (p < H) { *ra = DZ2 + p; *rb = -1; return; }
    p -= H;
    if (p < 4 * H) { *ra = D3 + p / H; *rb = H2 + p % H; return; }
    p -= 4 * H;
    *ra = D3 + p;
    *rb = -1;
}

__global__ __launch_bounds__(256) void k_mlp_partial(const float* __restrict__ rec, int64_t N, int64_t D, int H,
                                                     int P, const int32_t* __restrict__ drone_world,
                                                     const int32_t* __restrict__ gidx, int64_t chunk,
                                                     float* __restrict__ part) {
    extern __shared__ float tile[];   // [R][64]
    const int R = 17 + 4 * H;
    const int b = blockIdx.x, k = blockIdx.y, nb = gridDim.x;
    const int64_t lo = (int64_t)b * chunk, hi = min(N, lo + chunk);
    int ra[MLP_PER_THREAD], rb[MLP_PER_THREAD];
    float acc[MLP_PER_THREAD];
#pragma unroll
    for (int q = 0; q < MLP_PER_THREAD; ++q) {
        const int p = threadIdx.x + q * 256;
        ra[q] = 0;
        rb[q] = -1;
        if (p < P) mlp_param_rows(p, H, &ra[q], &rb[q]);
        acc[q] = 0.f;
    }
    for (int64_t n0 = lo; n0 < hi; n0 += 64) {
        for (int i = threadIdx.x; i < R * 64; i += 256) {
            const int r = i / 64, c = i % 64;
            const int64_t n = n0 + c;
            float v = 0.f;
            if (n < hi && gidx[drone_world[n % D]] == k) v = rec[(size_t)r * N + n];
            tile[r * 64 + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MLP_PER_THREAD; ++q) {
            if (threadIdx.x + q * 256 >= P) continue;
            const float* A = tile + ra[q] * 64;
            float s = 0.f;
            if (rb[q] < 0) {
                for (int c = 0; c < 64; ++c) s += A[c];
            } else {
                const float* Bv = tile + rb[q] * 64;
                for (int c = 0; c < 64; ++c) s = fmaf(A[c], Bv[c], s);
            }
            acc[q] += s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < MLP_PER_THREAD; ++q) {
        const int p = threadIdx.x + q * 256;
        if (p < P) part[((size_t)k * nb + b) * P + p] = acc[q];
    }
}

__global__ __launch_bounds__(256) void k_mlp_final(const float* __restrict__ part, int nb, int P,
                                                   float* __restrict__ g) {
    const int k = blockIdx.x;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        float s = 0.f;
        for (int b = 0; b < nb; ++b) s += part[((size_t)k * nb + b) * P + p];
        g[(size_t)k * P + p] = s;
    }
}

// workgroups per gain of the stage-1 reduction for D drones
static int gain_blocks(int64_t D) {
    const int64_t nb = (D + 511) / 512;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, GAIN_MAX_BLOCKS));
}

// Scratch of cf_rollout_backward_noalloc: one static device array, each GPU that
// runs the library holds its own copy until the process ends. Host code reaches
// it only through the address hipGetSymbolAddress gives per device (at
// cf_create); calls on one GPU share it.
static __device__ __align__(256) float scratch[CF_NOALLOC_SCRATCH_BYTES / sizeof(float)];
constexpr int MAX_SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[MAX_SCRATCH_DEVICES] = {};

// the scratch address of the current device h->device, looked up once per device
static hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) return hipSuccess;   // no static scratch there
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (float*)p;
    return hipSuccess;
}

static float* scratch_of(int dev) {
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// ---------------------------------------------------------------------------
// handle

namespace {

// part: 0 the whole launch sequence, MS_FP / MS_ID one model's launches of a
// mixed handle (captured and replayed separately, each on its own stream)
struct GraphKey {
    const void* st; const void* cmd; const void* nf; int k; int wq; int tile; int chunk; int plain; int waves;
    int part;
    bool operator<(const GraphKey& o) const {
        return std::tie(st, cmd, nf, k, wq, tile, chunk, plain, waves, part) <
               std::tie(o.st, o.cmd, o.nf, o.k, o.wq, o.tile, o.chunk, o.plain, o.waves, o.part);
    }
};

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
};

// Per-launch timing of the held-step kernels (CF_F_TIMING): an event pair around
// every kernel launch of a cf_step_k call, recorded on the stream the kernel is
// launched on (slot 0: the handle's stream, slot 1: the second per-model stream).
constexpr int MAX_TIMED = 512;
struct LaunchTimer {
    hipEvent_t a[MAX_TIMED] = {};
    hipEvent_t b[MAX_TIMED] = {};
    int n = 0;
    int made = 0;
};

}  // namespace

struct cf_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    hipStream_t aux_stream = nullptr;      // second stream for per-model launches (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int M = 0;
    int64_t D = 0;
    int S = 0;
    int models = 0;  // MS_*
    int control = 0, integ = 0, renorm = 1;
    float dt = 0.f;
    int ctrl_every = 1;              // onboard controller every n physics steps (1 without one)
    float dtc = 0.f, inv_dtc = 0.f;  // its period and inverse
    uint32_t flags = 0;
    int n_gains = 0;
    std::vector<int32_t> counts;
    std::vector<int64_t> offsets;
    std::vector<uint8_t> model_of_world;
    int cus = 256;
    std::string arch;
    // device copies
    float* par_aos = nullptr;
    float* par_soa = nullptr;
    int32_t* drone_world = nullptr;
    int64_t* d_offsets = nullptr;
    int32_t* d_gidx = nullptr;
    // tiles for the current tile size
    int4* tiles = nullptr;
    int n_tiles = 0;
    int n_tiles_fp = 0;  // tiles of first-principles worlds come first
    int tiles_for = 0;
    // packed tiles of the held-step kernels (tiles span worlds of one model) and
    // the drone list they index
    int4* ptiles = nullptr;
    int n_ptiles = 0;
    int n_ptiles_fp = 0;
    int ptiles_for = 0;
    int32_t* plist = nullptr;
    unsigned* counters = nullptr;
    int n_counters = 0;
    // launch choice
    int lane_ok = 0;     // all worlds one model: per-lane mapping possible
    int aero = 0;        // some world has propeller inertia, drag or a general rotor law
    int use_wq = 0;
    int tile = 64;
    int chunk = 0;       // 0 = all k steps in one launch
    int split = 1;       // mixed handles: one launch per model on two streams
    int wq_waves = 0;    // work queue: resident waves per compute unit of each launch (0 = all that fit)
    int mode = LM_TILE;
    // scratch
    DevBuf ref_tab, seg, ggc, rec, gpart, loss_tmp;
    // checkpoint tags: this handle's id, its count of forwards with a checkpoint
    // buffer, their tags by buffer, and a device word the backward kernels set
    // when a buffer no longer holds the tag the host matched
    uint32_t id = 0;
    uint32_t generation = 0;
    cfh::CkptRegistry ckpts;
    uint32_t* dflag = nullptr;
    cf_status sticky = CF_OK;
    std::map<GraphKey, hipGraphExec_t> graphs;
    LaunchTimer timers[2];
};

struct cf_mppi {
    cf_handle* h = nullptr;
    cfk::MppiArgs base{};
    cfk::KernelSel ks{};
    float* cost = nullptr;        // [C][N]
    float* elite_u = nullptr;     // [C][H*4][n_e]
    int32_t* elite_idx = nullptr; // [C][n_e]
    float* elite_cost = nullptr;  // [C][n_e]
    float* cost_min = nullptr;    // [C]
};

namespace {

cf_status from_hip(hipError_t e) {
    if (e == hipSuccess) return CF_OK;
    if (e == hipErrorOutOfMemory) return CF_ENOMEM;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return CF_ENODEV;
    return CF_EDEVICE;
}

cf_status note(cf_handle* h, hipError_t e) {
    cf_status s = from_hip(e);
    if (s == CF_EDEVICE && h->sticky == CF_OK) h->sticky = s;
    return s;
}

template <class T>
hipError_t dalloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    return hipMalloc((void**)p, n * sizeof(T));
}

hipError_t ensure(DevBuf& b, size_t bytes) {
    if (b.n >= bytes && b.p) return hipSuccess;
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
    hipError_t e = hipMalloc(&b.p, bytes ? bytes : 1);
    if (e == hipSuccess) b.n = bytes;
    return e;
}

// caller buffer check: ptr must be device memory holding at least `bytes`
cf_status check_dev(const void* ptr, size_t bytes) {
    if (!ptr) return CF_EINVAL;
    if (bytes == 0) return CF_OK;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) != hipSuccess) {
        (void)hipGetLastError();
        return CF_EINVAL;
    }
    const char* b = (const char*)base;
    const char* p = (const char*)ptr;
    if (p < b || (size_t)(p - b) + bytes > size) return CF_EINVAL;
    return CF_OK;
}

hipError_t build_tiles(cf_handle* h, int tile) {
    if (h->tiles && h->tiles_for == tile) return hipSuccess;
    int nfp = 0;
    const std::vector<cfh::Tile> v = cfh::tile_list(h->counts, h->offsets, h->model_of_world, h->control, tile, &nfp);
    std::vector<int4> dv(v.size());
    for (size_t i = 0; i < v.size(); ++i) dv[i] = make_int4(v[i].world, v[i].first, v[i].count, v[i].model);
    if (h->tiles) hipFree(h->tiles);
    h->tiles = nullptr;
    h->n_tiles = (int)dv.size();
    h->n_tiles_fp = nfp;
    hipError_t e = dalloc(&h->tiles, dv.size());
    if (e != hipSuccess) return e;
    if (!dv.empty()) e = hipMemcpy(h->tiles, dv.data(), dv.size() * sizeof(int4), hipMemcpyHostToDevice);
    h->tiles_for = tile;
    return e;
}

hipError_t build_packed_tiles(cf_handle* h, int tile) {
    if (h->ptiles && h->ptiles_for == tile) return hipSuccess;
    int nfp = 0;
    std::vector<int32_t> list;
    const std::vector<cfh::PackedTile> v =
        cfh::packed_tiles(h->counts, h->offsets, h->model_of_world, tile, &list, &nfp);
    hipError_t e = hipSuccess;
    if (!h->plist && !list.empty()) {
        if ((e = dalloc(&h->plist, list.size())) != hipSuccess) return e;
        if ((e = hipMemcpy(h->plist, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return e;
    }
    std::vector<int4> dv(v.size());
    for (size_t i = 0; i < v.size(); ++i) dv[i] = make_int4(v[i].first, v[i].count, v[i].model, 0);
    if (h->ptiles) hipFree(h->ptiles);
    h->ptiles = nullptr;
    h->n_ptiles = (int)dv.size();
    h->n_ptiles_fp = nfp;
    if ((e = dalloc(&h->ptiles, dv.size())) != hipSuccess) return e;
    if (!dv.empty()) e = hipMemcpy(h->ptiles, dv.data(), dv.size() * sizeof(int4), hipMemcpyHostToDevice);
    h->ptiles_for = tile;
    return e;
}

void clear_graphs(cf_handle* h) {
    for (auto& kv : h->graphs) hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

// Runs fn(models, tiles, n_tiles, stream, slot) over a tile list whose
// first-principles tiles come first: once for all tiles (uniform-model handles,
// or a single mixed launch), or once per model with the identified-model launch
// forked onto the auxiliary stream and joined back with events (also valid
// while capturing a graph).
template <class F>
hipError_t per_model_on(cf_handle* h, hipStream_t s, int split, const int4* tiles, int n, int n_fp, F&& fn) {
    if (!(h->models == MS_BOTH && split)) return fn(h->models, tiles, n, s, 0);
    hipError_t e;
    const int n_id = n - n_fp;
    if ((e = hipEventRecord(h->ev_fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(h->aux_stream, h->ev_fork, 0)) != hipSuccess) return e;
    if (n_fp > 0 && (e = fn(MS_FP, tiles, n_fp, s, 0)) != hipSuccess) return e;
    if (n_id > 0 && (e = fn(MS_ID, tiles + n_fp, n_id, h->aux_stream, 1)) != hipSuccess) return e;
    if ((e = hipEventRecord(h->ev_join, h->aux_stream)) != hipSuccess) return e;
    return hipStreamWaitEvent(s, h->ev_join, 0);
}

// over the per-world tiles (rollouts)
template <class F>
hipError_t per_model(cf_handle* h, hipStream_t s, int split, F&& fn) {
    return per_model_on(h, s, split, h->tiles, h->n_tiles, h->n_tiles_fp, fn);
}

// over the packed tiles (held steps); only = MS_FP or MS_ID: that model's tiles
// alone, on stream s (its slot: 0 first-principles, 1 identified)
template <class F>
hipError_t per_model_packed(cf_handle* h, hipStream_t s, int split, int only, F&& fn) {
    if (only == MS_FP) return h->n_ptiles_fp > 0 ? fn(MS_FP, h->ptiles, h->n_ptiles_fp, s, 0) : hipSuccess;
    if (only == MS_ID) {
        const int n_id = h->n_ptiles - h->n_ptiles_fp;
        return n_id > 0 ? fn(MS_ID, h->ptiles + h->n_ptiles_fp, n_id, s, 1) : hipSuccess;
    }
    return per_model_on(h, s, split, h->ptiles, h->n_ptiles, h->n_ptiles_fp, fn);
}

KernelSel selection(const cf_handle* h, int mode, int tile) {
    KernelSel ks;
    ks.models = h->models;
    ks.ctrl = h->control;
    ks.integ = h->integ;
    ks.mode = mode;
    ks.tile = tile;
    ks.aero = h->aero;
    return ks;
}

StepArgs step_args(const cf_handle* h, float* st, const float* cmd, int K, uint32_t* nf) {
    StepArgs a;
    a.st = st;
    a.cmd = cmd;
    a.D = h->D;
    a.M = h->M;
    a.par_aos = h->par_aos;
    a.par_soa = h->par_soa;
    a.drone_world = h->drone_world;
    a.dt = h->dt;
    a.dtc = h->dtc;
    a.inv_dtc = h->inv_dtc;
    a.ctrl_every = h->ctrl_every;
    a.renorm = h->renorm;
    a.K = K;
    a.nonfinite = (h->flags & CF_F_NONFINITE_CHECK) ? nf : nullptr;
    a.plist = h->plist;
    return a;
}

std::string cache_path() {
    const char* p = std::getenv("CFSIM_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/cfsim_autotune.txt";
}

std::string signature(const cf_handle* h) {
    char buf[256];
    int nfp = 0;
    for (auto m : h->model_of_world) nfp += (m == MODEL_FP);
    // every field that selects a different kernel or changes its work per step
    std::snprintf(buf, sizeof buf, "v3|%s|M%d|D%lld|fp%d|c%d|i%d|a%d|n%d", h->arch.c_str(), h->M, (long long)h->D,
                  nfp, h->control, h->integ, h->aero, h->ctrl_every);
    return buf;
}

void apply_choice(cf_handle* h, int wq, int tile, int chunk, int split) {
    if (tile != 64 && tile != 128 && tile != 256) tile = 64;
    h->split = split ? 1 : 0;
    h->use_wq = wq ? 1 : 0;
    h->tile = tile;
    h->chunk = chunk > 0 ? chunk : 0;
    h->mode = (h->lane_ok && !h->use_wq && h->D > 0 && (double)h->D / h->M < 32.0) ? LM_LANE : LM_TILE;
    clear_graphs(h);
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface

extern "C" {

const char* cf_strerror(cf_status s) {
    switch (s) {
        case CF_OK: return "success";
        case CF_EINVAL: return "invalid argument";
        case CF_ENODEV: return "no usable HIP device";
        case CF_ENOMEM: return "out of memory";
        case CF_EDEVICE: return "HIP device or runtime error";
        case CF_ESTATE: return "call sequence or checkpoint mismatch";
        case CF_EUNSUPPORTED: return "unsupported by this library";
        default: return "unknown status";
    }
}

cf_status cf_create(const cf_desc* d, cf_handle** out) {
    if (!out) return CF_EINVAL;
    *out = nullptr;
    std::vector<int32_t> counts, gidx;
    std::vector<uint8_t> models;
    int64_t D = 0;
    cf_status st = cfh::validate_desc(d, counts, models, gidx, &D);
    if (st != CF_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return CF_ENODEV;
    }
    int dev = d->device;
    if (dev < 0) {
        if (hipGetDevice(&dev) != hipSuccess) return CF_ENODEV;
    }
    if (dev >= ndev) return CF_ENODEV;
    if (hipSetDevice(dev) != hipSuccess) return CF_ENODEV;

    cf_handle* h = new (std::nothrow) cf_handle();
    if (!h) return CF_ENOMEM;
    h->device = dev;
    h->stream = (hipStream_t)d->stream;
    h->M = d->n_worlds;
    h->D = D;
    h->control = d->control;
    h->integ = d->integrator;
    h->renorm = d->renorm_q;
    h->dt = d->dt;
    h->flags = d->flags;
    h->n_gains = d->n_gains;
    h->counts = counts;
    h->model_of_world = models;
    h->offsets.assign(h->M + 1, 0);
    for (int w = 0; w < h->M; ++w) h->offsets[w + 1] = h->offsets[w] + counts[w];
    int has_fp = 0, has_id = 0;
    for (auto m : models) (m == CF_MODEL_FP ? has_fp : has_id) = 1;
    // only first-principles worlds behind the attitude, torque or position
    // interface have an onboard controller whose rate can differ
    h->ctrl_every = (has_fp && d->control != CF_CTRL_ROTOR && d->ctrl_every > 1) ? d->ctrl_every : 1;
    h->dtc = (float)((double)h->ctrl_every * (double)h->dt);
    h->inv_dtc = 1.0f / h->dtc;
    h->models = (has_fp ? MS_FP : 0) | (has_id ? MS_ID : 0);
    h->S = has_fp ? (h->control == CF_CTRL_ATT_PID ? CF_S_FP_PID : CF_S_FP_ROTOR) : CF_S_ID;
    h->lane_ok = (h->models != MS_BOTH);
    for (int w = 0; w < h->M; ++w) {
        const float* r = d->params + (size_t)w * CF_NPARAM;
        // the kernel variants with the full first-principles terms: rotor inertia,
        // drag, a rotor law beyond W' = c_v (W_cmd - W), or a drag-torque
        // polynomial that is not the thrust polynomial scaled
        double kap = 0.0;
        if (r[CF_P_DRAG] != 0.f || r[CF_P_DRAG + 1] != 0.f || r[CF_P_DRAG + 2] != 0.f ||
            (models[w] == CF_MODEL_FP &&
             (r[CF_P_JP] != 0.f || r[CF_P_MOTOR_UP + 1] != 0.f || r[CF_P_MOTOR_DOWN + 1] != 0.f ||
              r[CF_P_MOTOR_DOWN] != r[CF_P_MOTOR_UP] || !cfh::torque_proportional(r, &kap))))
            h->aero = 1;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        h->cus = prop.multiProcessorCount;
        h->arch = prop.gcnArchName;
        for (auto& c : h->arch)
            if (c == ':' || c == ' ') c = '_';
    }

    auto fail = [&](hipError_t e) {
        cf_status s = from_hip(e);
        cf_destroy(h);
        return s == CF_OK ? CF_EDEVICE : s;
    };
    hipError_t e;
    const size_t M = (size_t)h->M;
    std::vector<float> aos((size_t)NREC * M), soa((size_t)NREC * M);
    for (size_t w = 0; w < M; ++w) cfh::derive_record(d->params + w * CF_NPARAM, aos.data() + w * NREC);
    for (size_t w = 0; w < M; ++w)
        for (int i = 0; i < NREC; ++i) soa[(size_t)i * M + w] = aos[w * NREC + i];
    std::vector<int32_t> dw((size_t)std::max<int64_t>(D, 1));
    for (int w = 0; w < h->M; ++w)
        for (int64_t k = h->offsets[w]; k < h->offsets[w + 1]; ++k) dw[k] = w;
    if ((e = dalloc(&h->par_aos, M * NREC)) != hipSuccess) return fail(e);
    if ((e = dalloc(&h->par_soa, M * NREC)) != hipSuccess) return fail(e);
    if ((e = dalloc(&h->drone_world, (size_t)std::max<int64_t>(D, 1))) != hipSuccess) return fail(e);
    if ((e = dalloc(&h->d_offsets, M + 1)) != hipSuccess) return fail(e);
    if ((e = dalloc(&h->d_gidx, M)) != hipSuccess) return fail(e);
    if ((e = scratch_setup(dev)) != hipSuccess) return fail(e);
    static std::atomic<uint32_t> next_id{1};
    h->id = next_id.fetch_add(1);
    if ((e = dalloc(&h->dflag, 1)) != hipSuccess) return fail(e);
    if ((e = hipMemset(h->dflag, 0, sizeof(uint32_t))) != hipSuccess) return fail(e);
    h->n_counters = 4096;
    if ((e = dalloc(&h->counters, (size_t)h->n_counters)) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(h->par_aos, aos.data(), aos.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    if ((e = hipMemcpy(h->par_soa, soa.data(), soa.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    if ((e = hipMemcpy(h->drone_world, dw.data(), dw.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    if ((e = hipMemcpy(h->d_offsets, h->offsets.data(), (M + 1) * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    if ((e = hipMemcpy(h->d_gidx, gidx.data(), M * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    // streams beyond the caller's are created only where they are used (the
    // auxiliary stream for mixed handles here, the capture stream at the first
    // graph capture): with few hardware queues per process, every extra stream
    // raises the chance that two busy streams share one
    if (h->models == MS_BOTH &&
        (e = hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking)) != hipSuccess)
        return fail(e);
    if ((e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming)) != hipSuccess) return fail(e);
    if ((e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming)) != hipSuccess) return fail(e);

    int wq = (h->flags & CF_F_WORKQUEUE) ? 1 : 0, tile = 64, chunk = 0, split = 1;
    if (!(h->flags & CF_F_NO_AUTOTUNE_CACHE) && !(h->flags & CF_F_WORKQUEUE)) {
        cfh::LaunchChoice c;
        if (cfh::cache_lookup(cache_path(), signature(h), &c)) { wq = c.wq; tile = c.tile; chunk = c.chunk; split = c.split; }
    }
    if (h->flags & CF_F_SINGLE_LAUNCH) split = 0;
    apply_choice(h, wq, tile, chunk, split);
    if ((e = build_tiles(h, h->tile)) != hipSuccess) return fail(e);
    *out = h;
    return CF_OK;
}

cf_status cf_destroy(cf_handle* h) {
    if (!h) return CF_OK;
    hipSetDevice(h->device);
    if (h->stream) hipStreamSynchronize(h->stream);
    else hipDeviceSynchronize();
    clear_graphs(h);
    hipFree(h->par_aos);
    hipFree(h->par_soa);
    hipFree(h->drone_world);
    hipFree(h->d_offsets);
    hipFree(h->d_gidx);
    hipFree(h->tiles);
    hipFree(h->ptiles);
    hipFree(h->plist);
    hipFree(h->counters);
    hipFree(h->dflag);
    for (DevBuf* b : {&h->ref_tab, &h->seg, &h->ggc, &h->rec, &h->gpart, &h->loss_tmp})
        if (b->p) hipFree(b->p);
    if (h->capture_stream) hipStreamDestroy(h->capture_stream);
    if (h->aux_stream) {
        hipStreamSynchronize(h->aux_stream);
        hipStreamDestroy(h->aux_stream);
    }
    for (auto& T : h->timers)
        if (T.made)
            for (int i = 0; i < MAX_TIMED; ++i) {
                hipEventDestroy(T.a[i]);
                hipEventDestroy(T.b[i]);
            }
    if (h->ev_fork) hipEventDestroy(h->ev_fork);
    if (h->ev_join) hipEventDestroy(h->ev_join);
    delete h;
    return CF_OK;
}

cf_status cf_state_dim(const cf_handle* h, int32_t* S) {
    if (!h || !S) return CF_EINVAL;
    *S = h->S;
    return CF_OK;
}

cf_status cf_total_drones(const cf_handle* h, int64_t* D) {
    if (!h || !D) return CF_EINVAL;
    *D = h->D;
    return CF_OK;
}

cf_status cf_world_offsets(const cf_handle* h, int64_t* off) {
    if (!h || !off) return CF_EINVAL;
    std::memcpy(off, h->offsets.data(), (h->M + 1) * sizeof(int64_t));
    return CF_OK;
}

cf_status cf_set_stream(cf_handle* h, void* stream) {
    if (!h) return CF_EINVAL;
    h->stream = (hipStream_t)stream;
    return CF_OK;
}

cf_status cf_launch_config(const cf_handle* h, int32_t* use_wq, int32_t* tile, int32_t* chunk) {
    if (!h || !use_wq || !tile || !chunk) return CF_EINVAL;
    *use_wq = h->use_wq | (h->split && h->models == MS_BOTH ? 2 : 0);
    *tile = h->tile;
    *chunk = h->chunk;
    return CF_OK;
}

cf_status cf_set_launch_config(cf_handle* h, int32_t use_wq, int32_t tile, int32_t chunk, int32_t wq_waves) {
    if (!h || use_wq < 0 || use_wq > 3 || (tile != 64 && tile != 128 && tile != 256) || chunk < 0) return CF_EINVAL;
    if (chunk > 0 && chunk % h->ctrl_every != 0) return CF_EINVAL;
    if (wq_waves < 0 || wq_waves > 128) return CF_EINVAL;
    hipSetDevice(h->device);
    apply_choice(h, use_wq & 1, tile, chunk, (use_wq >> 1) & 1);
    h->wq_waves = wq_waves;
    return note(h, build_tiles(h, h->tile));
}

cf_status cf_launch_times(cf_handle* h, int32_t slot, float* ms, int32_t max_n, int32_t* n) {
    if (!h || !n || slot < 0 || slot > 1 || max_n < 0 || (max_n > 0 && !ms)) return CF_EINVAL;
    if (!(h->flags & CF_F_TIMING)) return CF_EINVAL;
    hipSetDevice(h->device);
    const LaunchTimer& T = h->timers[slot];
    const int m = std::min(T.n, (int)max_n);
    for (int i = 0; i < m; ++i) {
        hipError_t e = hipEventSynchronize(T.b[i]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], T.a[i], T.b[i]);
        if (e != hipSuccess) return note(h, e);
    }
    *n = T.n;
    return CF_OK;
}

cf_status cf_last_error(cf_handle* h) {
    if (!h) return CF_EINVAL;
    hipSetDevice(h->device);
    hipError_t e = h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize();
    if (e != hipSuccess) note(h, e);
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) note(h, e2);
    uint32_t flag = 0;
    if (h->sticky == CF_OK && hipMemcpy(&flag, h->dflag, sizeof flag, hipMemcpyDeviceToHost) == hipSuccess && flag)
        h->sticky = CF_ESTATE;
    return h->sticky;
}

cf_status cf_reset(cf_handle* h, float* state, const float* init, const uint8_t* world_mask) {
    if (!h) return CF_EINVAL;
    if (h->sticky != CF_OK) return h->sticky;
    if (h->D == 0) return CF_OK;
    const size_t bytes = (size_t)h->S * h->D * sizeof(float);
    if (check_dev(state, bytes) || check_dev(init, bytes)) return CF_EINVAL;
    if (world_mask && check_dev(world_mask, (size_t)h->M)) return CF_EINVAL;
    const char* s0 = (const char*)state;
    const char* i0 = (const char*)init;
    if (s0 < i0 + bytes && i0 < s0 + bytes) return CF_EINVAL;
    hipSetDevice(h->device);
    const unsigned grid = (unsigned)((h->D + 255) / 256);
    hipLaunchKernelGGL(k_reset, dim3(grid), dim3(256), 0, h->stream, state, init, h->S, h->D, h->drone_world,
                       world_mask);
    return note(h, hipGetLastError());
}

// CF_F_TIMING: the event before (end = 0) or after (end = 1) a kernel launch on
// stream st; the pairs of one cf_step_k call (or of the graph it captured)
static int slot_of(const cf_handle* h, hipStream_t st) { return (h->aux_stream && st == h->aux_stream) ? 1 : 0; }

static hipError_t timer_event(cf_handle* h, int slot, hipStream_t st, int end);

static hipError_t timer_mark(cf_handle* h, int slot, hipStream_t st, int end) {
    // launches captured into a graph are timed as a whole at each replay
    if (!(h->flags & CF_F_TIMING) || (h->flags & CF_F_GRAPH)) return hipSuccess;
    return timer_event(h, slot, st, end);
}

static hipError_t timer_event(cf_handle* h, int slot, hipStream_t st, int end) {
    LaunchTimer& T = h->timers[slot];
    if (T.n >= MAX_TIMED) return hipSuccess;   // launches beyond the capacity are not timed
    hipError_t e;
    if (!T.made) {
        for (int i = 0; i < MAX_TIMED; ++i) {
            if ((e = hipEventCreate(&T.a[i])) != hipSuccess) return e;
            if ((e = hipEventCreate(&T.b[i])) != hipSuccess) return e;
        }
        T.made = 1;
    }
    if (!end) return hipEventRecord(T.a[T.n], st);
    e = hipEventRecord(T.b[T.n], st);
    ++T.n;
    return e;
}

// enqueue k held-command steps with the current launch choice on stream s; only
// = MS_FP or MS_ID enqueues that model's launches alone, on s
static cf_status enqueue_steps(cf_handle* h, float* state, const float* cmd, int k, uint32_t* nf, hipStream_t s,
                               int plain, int only = 0) {
    hipError_t e = hipSuccess;
    if (!(h->flags & CF_F_GRAPH)) {
        h->timers[0].n = 0;
        h->timers[1].n = 0;
    }
    // the packed tiles of the current tile size (built before any graph capture
    // by cf_step_k, so this returns at once there)
    if ((e = build_packed_tiles(h, h->tile)) != hipSuccess) return note(h, e);
    const int n = h->ctrl_every;  // k is a multiple of n: every launch starts on a controller step
    if (plain) {
        // one step per launch; with a slower onboard controller, one controller
        // period per launch (its held commands are not part of the state)
        const int mode = h->mode == LM_LANE ? LM_LANE : LM_TILE;
        const StepArgs a = step_args(h, state, cmd, n, nf);
        e = per_model_packed(h, s, h->split, only, [&](int models, const int4* tiles, int nt, hipStream_t st, int) {
            KernelSel ks = selection(h, mode, h->tile);
            ks.models = models;
            hipError_t r = hipSuccess;
            for (int i = 0; i < k / n && r == hipSuccess; ++i) {
                if ((r = timer_mark(h, slot_of(h, st), st, 0)) != hipSuccess) break;
                r = launch_step(ks, a, tiles, nt, nullptr, 0, st);
                if (r == hipSuccess) r = timer_mark(h, slot_of(h, st), st, 1);
            }
            return r;
        });
        return note(h, e);
    }
    int chunk = (h->chunk > 0 && h->chunk < k) ? h->chunk : k;
    chunk = ((chunk + n - 1) / n) * n;
    const int n_launch = (k + chunk - 1) / chunk;
    // queue heads: one per launch, the first-principles launches' in the first half
    // of the counter array, the identified ones' in the second (a model's graph
    // clears only its own)
    const int half = h->n_counters / 2;
    if (h->use_wq) {
        if (n_launch > half) return CF_EINVAL;
        for (int slot = 0; slot < 2; ++slot) {
            if ((only == MS_FP && slot == 1) || (only == MS_ID && slot == 0)) continue;
            hipLaunchKernelGGL(k_fill_u32, dim3((n_launch + 255) / 256), dim3(256), 0, s, h->counters + slot * half,
                               n_launch, 0u);
            if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
        }
    }
    e = per_model_packed(h, s, h->split, only, [&](int models, const int4* tiles, int nt, hipStream_t st, int slot) {
        KernelSel ks = selection(h, h->use_wq ? LM_WQ : h->mode, h->tile);
        ks.models = models;
        int blocks = 0;
        if (h->use_wq) {
            int per_cu = step_wq_blocks_per_cu(ks);
            // a cap leaves SIMD registers to work on other streams (the overlapped adjoint)
            if (h->wq_waves > 0) per_cu = std::min(per_cu, std::max(1, h->wq_waves * 64 / ks.tile));
            blocks = std::max(1, std::min(nt, per_cu * h->cus));
        }
        hipError_t r = hipSuccess;
        for (int c = 0; c < n_launch && r == hipSuccess; ++c) {
            const int kk = std::min(chunk, k - c * chunk);
            const StepArgs a = step_args(h, state, cmd, kk, nf);
            if ((r = timer_mark(h, slot, st, 0)) != hipSuccess) break;
            r = launch_step(ks, a, tiles, nt, h->use_wq ? h->counters + slot * half + c : nullptr, blocks, st);
            if (r == hipSuccess) r = timer_mark(h, slot, st, 1);
        }
        return r;
    });
    return note(h, e);
}

cf_status cf_step_k(cf_handle* h, float* state, const float* cmd, int32_t k, uint32_t* nf) {
    if (!h || k < 1) return CF_EINVAL;
    if (k % h->ctrl_every != 0) return CF_EINVAL;
    if (h->sticky != CF_OK) return h->sticky;
    if (h->D == 0) return CF_OK;
    if (check_dev(state, (size_t)h->S * h->D * sizeof(float)) ||
        check_dev(cmd, (size_t)4 * h->D * sizeof(float)))
        return CF_EINVAL;
    if (nf && check_dev(nf, (size_t)h->M * sizeof(uint32_t))) return CF_EINVAL;
    hipSetDevice(h->device);
    hipError_t e = build_packed_tiles(h, h->tile);
    if (e != hipSuccess) return note(h, e);
    const int plain = (h->flags & CF_F_PLAIN_KERNEL) ? 1 : 0;
    if (!(h->flags & CF_F_GRAPH)) return enqueue_steps(h, state, cmd, k, nf, h->stream, plain);

    // a mixed handle with one launch per model keeps a graph per model and replays
    // them on its two streams, as the direct form runs them
    const bool two = h->models == MS_BOTH && h->split;
    hipGraphExec_t ge[2] = {nullptr, nullptr};
    for (int p = 0; p < (two ? 2 : 1); ++p) {
        const int part = two ? (p == 0 ? MS_FP : MS_ID) : 0;
        const GraphKey key{state, cmd, nf, k, h->use_wq * 2 + h->split, h->tile, h->chunk, plain, h->wq_waves, part};
        auto it = h->graphs.find(key);
        if (it == h->graphs.end()) {
            if (h->graphs.size() >= 64) {
                clear_graphs(h);
                if (p == 1) return cf_step_k(h, state, cmd, k, nf);   // the first model's graph was cleared too
            }
            if (!h->capture_stream &&
                (e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking)) != hipSuccess)
                return note(h, e);
            hipStream_t cs = h->capture_stream;
            if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return note(h, e);
            cf_status st = enqueue_steps(h, state, cmd, k, nf, cs, plain, part);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (st != CF_OK) {
                if (g) hipGraphDestroy(g);
                return st;
            }
            if (e2 != hipSuccess) return note(h, e2);
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) return note(h, e);
            it = h->graphs.emplace(key, x).first;
        }
        ge[p] = it->second;
    }
    // with CF_F_TIMING one event pair brackets the whole replay (slot 0)
    const bool timed = (h->flags & CF_F_TIMING) != 0;
    h->timers[0].n = 0;
    h->timers[1].n = 0;
    if (timed && (e = timer_event(h, 0, h->stream, 0)) != hipSuccess) return note(h, e);
    if (two) {
        if ((e = hipEventRecord(h->ev_fork, h->stream)) != hipSuccess) return note(h, e);
        if ((e = hipStreamWaitEvent(h->aux_stream, h->ev_fork, 0)) != hipSuccess) return note(h, e);
        if ((e = hipGraphLaunch(ge[0], h->stream)) != hipSuccess) return note(h, e);
        if ((e = hipGraphLaunch(ge[1], h->aux_stream)) != hipSuccess) return note(h, e);
        if ((e = hipEventRecord(h->ev_join, h->aux_stream)) != hipSuccess) return note(h, e);
        if ((e = hipStreamWaitEvent(h->stream, h->ev_join, 0)) != hipSuccess) return note(h, e);
    } else if ((e = hipGraphLaunch(ge[0], h->stream)) != hipSuccess) {
        return note(h, e);
    }
    if (timed && (e = timer_event(h, 0, h->stream, 1)) != hipSuccess) return note(h, e);
    return CF_OK;
}

// ---------------------------------------------------------------------------
// rollout

static int roll_mode(const cf_handle* h) {
    return (h->lane_ok && h->D > 0 && (double)h->D / h->M < 32.0) ? LM_LANE : LM_TILE;
}

// ref_tab_buf: device [(T + 1)][6] for the figure-eight table, or null to use the
// handle's own (grown on demand)
static cf_status prepare_objective(cf_handle* h, const cf_objective* obj, int T, RollArgs& a,
                                   float* ref_tab_buf = nullptr) {
    a.has_obj = obj ? 1 : 0;
    a.gain = nullptr;
    a.gidx = h->d_gidx;
    a.ref_tab = nullptr;
    a.ref_user = 0;
    a.ref_off = nullptr;
    a.ref_shift = nullptr;
    a.squash = 0;
    a.w_u = 0.f;
    a.obj_kind = 0;
    a.ubuf = nullptr;
    if (!obj) return CF_OK;
    if (!(std::isfinite(obj->w_u) && obj->w_u >= 0.f)) return CF_EINVAL;
    if (obj->kind != CF_OBJ_TRACKING && obj->kind != CF_OBJ_BPTT_REWARD) return CF_EINVAL;
    if (obj->kind == CF_OBJ_BPTT_REWARD) {
        if (h->control == CF_CTRL_POSITION && (h->models & MS_FP)) return CF_EINVAL;
        bool ok = std::isfinite(obj->w_tilt) && obj->w_tilt >= 0.f;
        for (int i = 0; i < 4; ++i) {
            ok = ok && std::isfinite(obj->w_act[i]) && obj->w_act[i] >= 0.f;
            ok = ok && std::isfinite(obj->w_dact[i]) && obj->w_dact[i] >= 0.f;
        }
        if (!ok) return CF_EINVAL;
        a.obj_kind = 1;
        a.w_tilt = obj->w_tilt;
        for (int i = 0; i < 4; ++i) {
            a.w_act[i] = obj->w_act[i];
            a.w_dact[i] = obj->w_dact[i];
        }
    }
    a.mlp_H = 0;
    a.mlp_P = 0;
    a.n_pol = 0;
    a.mlp_rec = nullptr;
    if (obj->policy_hidden < 0 || obj->policy_hidden > CF_MLP_MAX_HIDDEN) return CF_EINVAL;
    if (obj->policy_hidden > 0) {
        const int H = obj->policy_hidden, P = CF_MLP_PARAMS(H);
        if (!obj->gain || h->n_gains < 1) return CF_EINVAL;
        if (check_dev(obj->gain, (size_t)h->n_gains * P * sizeof(float))) return CF_EINVAL;
        // policies and each lane's activations in LDS; tiles of 64 lanes
        if (((size_t)h->n_gains * P + (size_t)4 * 64 * H) * sizeof(float) > 65536) return CF_EUNSUPPORTED;
        if (roll_mode(h) == LM_TILE && h->tile != 64) return CF_EUNSUPPORTED;
        a.mlp_H = H;
        a.mlp_P = P;
        a.n_pol = h->n_gains;
        a.gain = obj->gain;
    } else if (obj->gain) {
        if (h->n_gains < 1) return CF_EINVAL;
        if (check_dev(obj->gain, (size_t)h->n_gains * 52 * sizeof(float))) return CF_EINVAL;
        a.gain = obj->gain;
    }
    if (obj->ref_offset) {
        if (check_dev(obj->ref_offset, (size_t)3 * h->D * sizeof(float))) return CF_EINVAL;
        a.ref_off = obj->ref_offset;
    }
    a.w_u = obj->w_u;
    {
        bool any = false, ok = true;
        for (int i = 0; i < 4; ++i) {
            ok = ok && std::isfinite(obj->policy_scale[i]) && obj->policy_scale[i] >= 0.f;
            any = any || obj->policy_scale[i] > 0.f;
        }
        if (!ok) return CF_EINVAL;
        if (any) {
            a.squash = 1;
            for (int i = 0; i < 4; ++i) a.act_s[i] = obj->policy_scale[i];
        }
    }
    if (obj->ref_time_shift) {
        // the shift moves the analytic figure-eight; a user table has no such form
        if (obj->ref_table) return CF_EINVAL;
        if (check_dev(obj->ref_time_shift, (size_t)h->D * sizeof(float))) return CF_EINVAL;
        a.ref_shift = obj->ref_time_shift;
    }
    if (obj->ref_table) {
        if (check_dev(obj->ref_table, (size_t)(T + 1) * 13 * sizeof(float))) return CF_EINVAL;
        a.ref_tab = obj->ref_table;
        a.ref_user = 1;
    } else {
        if (!(std::isfinite(obj->ref_period) && obj->ref_period > 0.f) || !std::isfinite(obj->ref_amp) ||
            obj->ref_step0 < 0)
            return CF_EINVAL;
        hipError_t e = hipSuccess;
        float* tab = ref_tab_buf;
        if (!tab) {
            if ((e = ensure(h->ref_tab, (size_t)(T + 1) * 6 * sizeof(float))) != hipSuccess) return note(h, e);
            tab = (float*)h->ref_tab.p;
        }
        hipLaunchKernelGGL(k_eight_table, dim3((T + 1 + 255) / 256), dim3(256), 0, h->stream, tab, T, h->dt,
                           obj->ref_amp, obj->ref_period, obj->ref_step0);
        if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
        a.ref_tab = tab;
        const double w0 = 2.0 * 3.14159265358979323846 / (double)obj->ref_period;
        a.ref_w = (float)w0;
        a.ref_inv_w = (float)(1.0 / w0);
    }
    return CF_OK;
}

static RollArgs roll_args(const cf_handle* h, const float* x0, const float* cmds, int T, int K) {
    RollArgs a;
    std::memset(&a, 0, sizeof a);
    a.x0 = x0;
    a.S_h = h->S;
    a.cmds = cmds;
    a.T = T;
    a.D = h->D;
    a.M = h->M;
    a.par_aos = h->par_aos;
    a.par_soa = h->par_soa;
    a.drone_world = h->drone_world;
    a.dt = h->dt;
    a.dtc = h->dtc;
    a.inv_dtc = h->inv_dtc;
    a.ctrl_every = h->ctrl_every;
    a.renorm = h->renorm;
    a.K = K;
    return a;
}


cf_status cf_ckpt_floats(const cf_handle* h, int32_t T, int32_t K, int32_t kind, int64_t* n) {
    if (!h || !n || T < 1 || K < 1) return CF_EINVAL;
    if (kind != CF_OBJ_TRACKING && kind != CF_OBJ_BPTT_REWARD) return CF_EINVAL;
    *n = cfh::ckpt_floats(T, K, h->S, h->D, kind);
    return CF_OK;
}

cf_status cf_rollout(cf_handle* h, const float* x0, const float* cmds, int32_t T, const cf_objective* obj,
                     int32_t K, float* ckpt, float* x_T, float* traj, float* loss, float* loss_world) {
    if (!h || T < 1 || K < 1) return CF_EINVAL;
    if (K % h->ctrl_every != 0 && h->ctrl_every % K != 0) return CF_EINVAL;
    if (h->sticky != CF_OK) return h->sticky;
    if (!obj && (loss || loss_world)) return CF_EINVAL;
    if (obj && obj->kind != CF_OBJ_TRACKING && obj->kind != CF_OBJ_BPTT_REWARD) return CF_EINVAL;
    const int kind = obj ? obj->kind : CF_OBJ_TRACKING;
    const size_t SD = (size_t)h->S * h->D * sizeof(float);
    if (h->D > 0) {
        if (check_dev(x0, SD) || check_dev(cmds, (size_t)T * 4 * h->D * sizeof(float))) return CF_EINVAL;
        if (ckpt && check_dev(ckpt, (size_t)cfh::ckpt_floats(T, K, h->S, h->D, kind) * sizeof(float)))
            return CF_EINVAL;
        if (x_T && check_dev(x_T, SD)) return CF_EINVAL;
        if (traj && check_dev(traj, (size_t)(T + 1) * SD)) return CF_EINVAL;
        if (loss && check_dev(loss, (size_t)h->D * sizeof(float))) return CF_EINVAL;
    }
    if (loss_world && check_dev(loss_world, (size_t)h->M * sizeof(float))) return CF_EINVAL;
    hipSetDevice(h->device);
    RollArgs a = roll_args(h, x0, cmds, T, K);
    cf_status st = prepare_objective(h, obj, T, a);
    if (st != CF_OK) return st;
    a.ckpt = ckpt;
    if (ckpt && a.obj_kind == 1) a.ubuf = ckpt + cfh::ckpt_ubuf_offset(T, K, h->S, h->D);
    a.xT = x_T;
    a.traj = traj;
    a.loss = loss;
    a.nonfinite = nullptr;
    hipError_t e = hipSuccess;
    if (loss_world && !loss) {
        if ((e = ensure(h->loss_tmp, (size_t)std::max<int64_t>(h->D, 1) * sizeof(float))) != hipSuccess)
            return note(h, e);
        a.loss = (float*)h->loss_tmp.p;
    }
    if (h->D > 0) {
        const int mode = roll_mode(h);
        if (mode == LM_TILE && (e = build_tiles(h, h->tile)) != hipSuccess) return note(h, e);
        e = per_model(h, h->stream, h->split, [&](int models, const int4* tiles, int nt, hipStream_t st, int) {
            KernelSel ks = selection(h, mode, mode == LM_LANE ? 64 : h->tile);
            ks.models = models;
            return launch_rollout_fwd(ks, a, tiles, nt, st);
        });
        if (e != hipSuccess) return note(h, e);
    }
    if (loss_world) {
        hipLaunchKernelGGL(k_reduce_world, dim3(h->M), dim3(256), 0, h->stream, a.loss, 1, h->D, h->d_offsets,
                           loss_world);
        if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
    }
    if (ckpt) {
        const cfh::CkptTag tag = cfh::make_tag(h->id, ++h->generation, T, K, h->S, h->D, obj);
        if (h->D > 0) {
            TagWords tw;
            std::memcpy(tw.w, tag.w, sizeof tw.w);
            uint32_t* dst = (uint32_t*)(ckpt + cfh::ckpt_tag_offset(T, K, h->S, h->D, kind));
            hipLaunchKernelGGL(k_write_tag, dim3(1), dim3(64), 0, h->stream, dst, tw);
            if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
        }
        h->ckpts.record(ckpt, tag);
    }
    return CF_OK;
}

// Device scratch of one backward call: the handle's buffers (grown on demand) or,
// without allocation, consecutive 256-byte-aligned slices of the static array.
struct BwdScratch {
    float* ref_tab = nullptr;   // [T + 1][6], figure-eight objectives
    float* seg = nullptr;       // [slots][S][D] recomputed segment states
    float* ggc = nullptr;       // [52][D] per-drone gain-gradient contributions
    float* rec = nullptr;       // MLP policy: [17 + 4 H][T][D] per-step records
    float* gpart = nullptr;     // [n_gains][blocks][52 or P] stage-1 sums
};

static cf_status rollout_backward_impl(cf_handle* h, const float* cmds, int32_t T, const cf_objective* obj,
                                       int32_t K, const float* ckpt, const float* dloss, float* g_cmds, float* g_x0,
                                       float* g_gain, bool noalloc) {
    if (!h || T < 1 || K < 1 || !ckpt) return CF_EINVAL;
    if (K % h->ctrl_every != 0 && h->ctrl_every % K != 0) return CF_EINVAL;
    if (h->sticky != CF_OK) return h->sticky;
    if (g_gain && (!obj || !obj->gain)) return CF_EINVAL;
    if (obj && obj->kind != CF_OBJ_TRACKING && obj->kind != CF_OBJ_BPTT_REWARD) return CF_EINVAL;
    const int kind = obj ? obj->kind : CF_OBJ_TRACKING;
    cfh::CkptTag tag;
    if (h->ckpts.match(ckpt, T, K, h->S, h->D, obj, &tag) != CF_OK) return CF_ESTATE;
    const size_t SD = (size_t)h->S * h->D * sizeof(float);
    if (h->D > 0) {
        if (check_dev(cmds, (size_t)T * 4 * h->D * sizeof(float))) return CF_EINVAL;
        if (check_dev(ckpt, (size_t)cfh::ckpt_floats(T, K, h->S, h->D, kind) * sizeof(float))) return CF_EINVAL;
        if (dloss && check_dev(dloss, (size_t)h->D * sizeof(float))) return CF_EINVAL;
        if (g_cmds && check_dev(g_cmds, (size_t)T * 4 * h->D * sizeof(float))) return CF_EINVAL;
        if (g_x0 && check_dev(g_x0, SD)) return CF_EINVAL;
    }
    const int Hp = obj ? obj->policy_hidden : 0;   // MLP policy width (validated below)
    if (Hp < 0 || Hp > CF_MLP_MAX_HIDDEN) return CF_EINVAL;
    const int Pp = Hp > 0 ? CF_MLP_PARAMS(Hp) : 52;
    if (g_gain && check_dev(g_gain, (size_t)h->n_gains * Pp * sizeof(float))) return CF_EINVAL;
    // scratch sizes (floats)
    const int64_t Dm = std::max<int64_t>(h->D, 1);
    // segment slots 1..K-1 hold recomputed states (slot 0 is the checkpoint itself);
    // with the reward objective slot K holds the final state of the last segment
    const int slots = std::min(K, T) + (kind == CF_OBJ_BPTT_REWARD ? 1 : 0);
    const int nb = gain_blocks(h->D);
    const size_t n_tab = (obj && !obj->ref_table) ? (size_t)(T + 1) * 6 : 0;
    const size_t n_seg = slots > 1 ? (size_t)slots * h->S * Dm : 0;
    const int64_t N_rec = (int64_t)T * Dm;
    const int nb_mlp = (int)std::max<int64_t>(1, std::min<int64_t>((N_rec + 2047) / 2048, GAIN_MAX_BLOCKS));
    const size_t n_ggc = (g_gain && Hp == 0) ? (size_t)52 * Dm : 0;
    const size_t n_rec = (g_gain && Hp > 0) ? (size_t)(17 + 4 * Hp) * N_rec : 0;
    const size_t n_part = !g_gain ? 0
                                  : (Hp > 0 ? (size_t)h->n_gains * nb_mlp * Pp : (size_t)h->n_gains * nb * GAIN_COMP);
    hipSetDevice(h->device);
    hipError_t e;
    BwdScratch sc;
    if (noalloc) {
        float* base = scratch_of(h->device);
        if (!base) return CF_EUNSUPPORTED;
        // 256-byte-aligned slices; sizes beyond the array are refused before any work
        auto up = [](size_t n) { return (n + 63) / 64 * 64; };
        const size_t cap = CF_NOALLOC_SCRATCH_BYTES / sizeof(float);
        if (up(n_tab) + up(n_seg) + up(n_ggc) + up(n_rec) + up(n_part) > cap) return CF_EINVAL;
        float* q = base;
        auto take = [&](size_t n) -> float* {
            if (n == 0) return nullptr;
            float* r = q;
            q += up(n);
            return r;
        };
        sc.ref_tab = take(n_tab);
        sc.seg = take(n_seg);
        sc.ggc = take(n_ggc);
        sc.rec = take(n_rec);
        sc.gpart = take(n_part);
    } else {
        if (n_seg && (e = ensure(h->seg, n_seg * sizeof(float))) != hipSuccess) return note(h, e);
        if (n_ggc && (e = ensure(h->ggc, n_ggc * sizeof(float))) != hipSuccess) return note(h, e);
        if (n_rec && (e = ensure(h->rec, n_rec * sizeof(float))) != hipSuccess) return note(h, e);
        if (n_part && (e = ensure(h->gpart, n_part * sizeof(float))) != hipSuccess) return note(h, e);
        sc.seg = (float*)h->seg.p;
        sc.ggc = (float*)h->ggc.p;
        sc.rec = (float*)h->rec.p;
        sc.gpart = (float*)h->gpart.p;
        sc.ref_tab = nullptr;   // prepare_objective uses the handle's table
    }
    RollArgs a = roll_args(h, nullptr, cmds, T, K);
    cf_status st = prepare_objective(h, obj, T, a, sc.ref_tab);
    if (st != CF_OK) return st;
    a.ckpt_in = ckpt;
    if (a.obj_kind == 1) a.ubuf = const_cast<float*>(ckpt) + cfh::ckpt_ubuf_offset(T, K, h->S, h->D);
    a.tag_in = (const uint32_t*)(ckpt + cfh::ckpt_tag_offset(T, K, h->S, h->D, kind));
    std::memcpy(a.tag_exp, tag.w, sizeof a.tag_exp);
    a.dflag = h->dflag;
    a.dloss = dloss;
    a.g_cmds = g_cmds;
    a.g_x0 = g_x0;
    a.seg = n_seg ? sc.seg : nullptr;
    a.ggc = (g_gain && Hp == 0) ? sc.ggc : nullptr;
    a.mlp_rec = (g_gain && Hp > 0) ? sc.rec : nullptr;
    if (h->D > 0) {
        const int mode = roll_mode(h);
        if (mode == LM_TILE && (e = build_tiles(h, h->tile)) != hipSuccess) return note(h, e);
        e = per_model(h, h->stream, h->split, [&](int models, const int4* tiles, int nt, hipStream_t st, int) {
            KernelSel ks = selection(h, mode, mode == LM_LANE ? 64 : h->tile);
            ks.models = models;
            return launch_rollout_bwd(ks, a, tiles, nt, st);
        });
        if (e != hipSuccess) return note(h, e);
    }
    if (g_gain && Hp > 0) {
        if (h->D > 0) {
            const int64_t chunk = (N_rec + nb_mlp - 1) / nb_mlp;
            hipLaunchKernelGGL(k_mlp_partial, dim3(nb_mlp, h->n_gains), dim3(256),
                               (size_t)(17 + 4 * Hp) * 64 * sizeof(float), h->stream, (const float*)sc.rec,
                               (int64_t)T * h->D, h->D, Hp, Pp, h->drone_world, h->d_gidx, chunk, sc.gpart);
            if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
            hipLaunchKernelGGL(k_mlp_final, dim3(h->n_gains), dim3(256), 0, h->stream, (const float*)sc.gpart,
                               nb_mlp, Pp, g_gain);
        } else {
            hipLaunchKernelGGL(k_fill_u32, dim3((h->n_gains * Pp + 255) / 256), dim3(256), 0, h->stream,
                               (unsigned*)g_gain, h->n_gains * Pp, 0u);
        }
        if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
    } else if (g_gain) {
        if (h->D > 0) {
            const int64_t chunk = (h->D + nb - 1) / nb;
            hipLaunchKernelGGL(k_gain_partial, dim3(nb, h->n_gains), dim3(256), 0, h->stream, (const float*)sc.ggc,
                               h->D, h->drone_world, h->d_gidx, chunk, sc.gpart);
            if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
            hipLaunchKernelGGL(k_gain_final, dim3(h->n_gains), dim3(64), 0, h->stream, (const float*)sc.gpart, nb,
                               g_gain);
        } else {
            hipLaunchKernelGGL(k_fill_u32, dim3((h->n_gains * 52 + 255) / 256), dim3(256), 0, h->stream,
                               (unsigned*)g_gain, h->n_gains * 52, 0u);
        }
        if ((e = hipGetLastError()) != hipSuccess) return note(h, e);
    }
    return CF_OK;
}

cf_status cf_rollout_backward(cf_handle* h, const float* x0, const float* cmds, int32_t T, const cf_objective* obj,
                              int32_t K, const float* ckpt, const float* dloss, float* g_cmds, float* g_x0,
                              float* g_gain) {
    (void)x0;   // the checkpoint holds it
    return rollout_backward_impl(h, cmds, T, obj, K, ckpt, dloss, g_cmds, g_x0, g_gain, false);
}

cf_status cf_rollout_backward_noalloc(cf_handle* h, const float* x0, const float* cmds, int32_t T,
                                      const cf_objective* obj, int32_t K, const float* ckpt, const float* dloss,
                                      float* g_cmds, float* g_x0, float* g_gain) {
    (void)x0;
    return rollout_backward_impl(h, cmds, T, obj, K, ckpt, dloss, g_cmds, g_x0, g_gain, true);
}


// ---------------------------------------------------------------------------
// autotune

cf_status cf_autotune(cf_handle* h, const float* state, const float* cmd, int32_t k, int32_t budget_ms) {
    if (!h || k < 1 || budget_ms < 1) return CF_EINVAL;
    if (h->sticky != CF_OK) return h->sticky;
    if (h->D == 0) return CF_OK;
    const size_t SD = (size_t)h->S * h->D * sizeof(float);
    if (check_dev(state, SD) || check_dev(cmd, (size_t)4 * h->D * sizeof(float))) return CF_EINVAL;
    hipSetDevice(h->device);
    float* work = nullptr;
    hipError_t e = hipMalloc(&work, SD);
    if (e != hipSuccess) return note(h, e);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    struct Cand { int wq, tile, chunk, split; };
    std::vector<Cand> cands;
    for (int split = 1; split >= (h->models == MS_BOTH ? 0 : 1); --split)
        for (int wq = 0; wq < 2; ++wq)
            for (int tile : {64, 128, 256})
                for (int chunk : {0, 100, 25}) {
                    if (chunk && chunk >= k) continue;
                    cands.push_back({wq, tile, chunk, split});
                }
    const int save_wq = h->use_wq, save_tile = h->tile, save_chunk = h->chunk, save_split = h->split;
    h->wq_waves = 0;   // candidates run with every wave that fits
    const uint32_t save_flags = h->flags;
    h->flags &= ~(CF_F_PLAIN_KERNEL | CF_F_GRAPH);
    float best = 1e30f;
    Cand bc{save_wq, save_tile, save_chunk, save_split};
    double spent = 0.0;
    cf_status st = CF_OK;
    for (const Cand& c : cands) {
        if (spent > budget_ms && best < 1e30f) break;
        apply_choice(h, c.wq, c.tile, c.chunk, c.split);
        if ((e = build_tiles(h, h->tile)) != hipSuccess) { st = note(h, e); break; }
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hipMemcpyAsync(work, state, SD, hipMemcpyDeviceToDevice, h->stream);
            hipEventRecord(e0, h->stream);
            st = enqueue_steps(h, work, cmd, k, nullptr, h->stream, 0);
            hipEventRecord(e1, h->stream);
            if (st != CF_OK) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = note(h, e); break; }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            spent += ms;
            ms_best = std::min(ms_best, ms);
        }
        if (st != CF_OK) break;
        if (ms_best < best) { best = ms_best; bc = c; }
    }
    h->flags = save_flags;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(work);
    if (st != CF_OK) {
        apply_choice(h, save_wq, save_tile, save_chunk, save_split);
        return st;
    }
    apply_choice(h, bc.wq, bc.tile, bc.chunk, bc.split);
    if ((e = build_tiles(h, h->tile)) != hipSuccess) return note(h, e);
    cfh::LaunchChoice lc;
    lc.wq = bc.wq; lc.tile = bc.tile; lc.chunk = bc.chunk; lc.split = bc.split; lc.ms = best;
    cfh::cache_store(cache_path(), signature(h), lc);
    return CF_OK;
}

// ---- sampled-rollout controller -------------------------------------------------

static void mppi_free(cf_mppi* m) {
    hipFree(m->cost);
    hipFree(m->elite_u);
    hipFree(m->elite_idx);
    hipFree(m->elite_cost);
    hipFree(m->cost_min);
}

cf_status cf_mppi_create(cf_handle* h, const cf_mppi_desc* d, cf_mppi** out) {
    if (!out) return CF_EINVAL;
    *out = nullptr;
    if (!h || !d) return CF_EINVAL;
    if (h->M != 1) return CF_EINVAL;
    if (d->n_controllers < 1 || d->n_samples < 1 || d->horizon < 1 || d->substeps < 1) return CF_EINVAL;
    if (d->n_controllers > 65535) return CF_EINVAL;  // grid y dimension of the rollout
    if ((int64_t)d->n_controllers * d->n_samples > 2147483647LL) return CF_EINVAL;
    if ((int64_t)d->n_controllers * d->horizon * 4 > 2147483647LL) return CF_EINVAL;
    if (d->n_elite < 1 || d->n_elite > d->n_samples || d->n_elite > cfk::MPPI_MAX_ELITE) return CF_EINVAL;
    if (!(std::isfinite(d->beta) && d->beta >= 0.f && d->beta < 1.f)) return CF_EINVAL;
    if (!(std::isfinite(d->lambda) && d->lambda > 0.f)) return CF_EINVAL;
    for (int i = 0; i < 4; ++i) {
        if (!(std::isfinite(d->sigma[i]) && d->sigma[i] >= 0.f)) return CF_EINVAL;
        if (!(std::isfinite(d->u_lo[i]) && std::isfinite(d->u_hi[i]) && d->u_lo[i] <= d->u_hi[i])) return CF_EINVAL;
        if (!(std::isfinite(d->u_ref[i]) && std::isfinite(d->r_u[i]) && d->r_u[i] >= 0.f)) return CF_EINVAL;
    }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(d->goal[i])) return CF_EINVAL;
    if (!(std::isfinite(d->q_p) && d->q_p >= 0.f && std::isfinite(d->q_v) && d->q_v >= 0.f &&
          std::isfinite(d->w_obs) && d->w_obs >= 0.f))
        return CF_EINVAL;
    if (d->n_obstacles < 0 || d->n_obstacles > CF_MPPI_MAX_OBSTACLES) return CF_EINVAL;
    for (int o = 0; o < d->n_obstacles; ++o) {
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(d->obstacles[o][i])) return CF_EINVAL;
        if (!(std::isfinite(d->obstacles[o][3]) && d->obstacles[o][3] > 0.f)) return CF_EINVAL;
    }
    if (h->sticky != CF_OK) return h->sticky;
    hipSetDevice(h->device);
    cf_mppi* m = new (std::nothrow) cf_mppi();
    if (!m) return CF_ENOMEM;
    m->h = h;
    cfk::MppiArgs& a = m->base;
    a.par = h->par_aos;
    a.C = d->n_controllers;
    a.N = d->n_samples;
    a.H = d->horizon;
    a.sub = d->substeps;
    a.n_e = d->n_elite;
    a.dt = h->dt;
    a.dtc = h->dtc;
    a.inv_dtc = h->inv_dtc;
    a.ctrl_every = h->ctrl_every;
    a.renorm = h->renorm;
    for (int i = 0; i < 4; ++i) {
        a.sigma[i] = d->sigma[i];
        a.u_lo[i] = d->u_lo[i];
        a.u_hi[i] = d->u_hi[i];
        a.u_ref[i] = d->u_ref[i];
        a.r_u[i] = d->r_u[i];
    }
    a.beta = d->beta;
    a.beta_c = (float)std::sqrt(1.0 - (double)d->beta * (double)d->beta);
    a.inv_lambda = (float)(1.0 / (double)d->lambda);
    for (int i = 0; i < 3; ++i) a.goal[i] = d->goal[i];
    a.q_p = d->q_p;
    a.q_v = d->q_v;
    a.w_obs = d->w_obs;
    a.n_obs = d->n_obstacles;
    for (int o = 0; o < d->n_obstacles; ++o) {
        for (int i = 0; i < 3; ++i) a.obs[o][i] = d->obstacles[o][i];
        const double r = d->obstacles[o][3];
        a.obs[o][3] = (float)(1.0 / (r * r));
    }
    a.seed = d->seed;
    m->ks = selection(h, LM_LANE, 256);
    const size_t CN = (size_t)a.C * a.N, CE = (size_t)a.C * a.n_e;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = dalloc(&m->cost, CN);
    if (e == hipSuccess) e = dalloc(&m->elite_u, CE * a.H * 4);
    if (e == hipSuccess) e = dalloc(&m->elite_idx, CE);
    if (e == hipSuccess) e = dalloc(&m->elite_cost, CE);
    if (e == hipSuccess) e = dalloc(&m->cost_min, (size_t)a.C);
    if (e != hipSuccess) {
        mppi_free(m);
        delete m;
        return from_hip(e);
    }
    *out = m;
    return CF_OK;
}

cf_status cf_mppi_destroy(cf_mppi* m) {
    if (!m) return CF_OK;
    hipSetDevice(m->h->device);
    if (m->h->stream) hipStreamSynchronize(m->h->stream);
    else hipDeviceSynchronize();
    mppi_free(m);
    delete m;
    return CF_OK;
}

cf_status cf_mppi_step(cf_mppi* m, const float* x_now, float* mean, int32_t shift, uint64_t iteration,
                       float* u_apply, int32_t* best, float* cost, int32_t* elite_idx, float* cost_min) {
    if (!m || shift < 0) return CF_EINVAL;
    cf_handle* h = m->h;
    if (h->sticky != CF_OK) return h->sticky;
    const cfk::MppiArgs& b = m->base;
    const size_t CN = (size_t)b.C * b.N, CE = (size_t)b.C * b.n_e;
    if (check_dev(x_now, (size_t)h->S * sizeof(float)) ||
        check_dev(mean, (size_t)b.C * b.H * 4 * sizeof(float)))
        return CF_EINVAL;
    if ((u_apply && check_dev(u_apply, 4 * sizeof(float))) || (best && check_dev(best, sizeof(int32_t))) ||
        (cost && check_dev(cost, CN * sizeof(float))) || (elite_idx && check_dev(elite_idx, CE * sizeof(int32_t))) ||
        (cost_min && check_dev(cost_min, (size_t)b.C * sizeof(float))))
        return CF_EINVAL;
    hipSetDevice(h->device);
    cfk::MppiArgs a = b;
    a.x_now = x_now;
    a.mean = mean;
    a.mean_out = mean;
    a.shift = shift;
    a.iter = iteration;
    a.cost = cost ? cost : m->cost;
    a.elite_u = m->elite_u;
    a.elite_idx = elite_idx ? elite_idx : m->elite_idx;
    a.elite_cost = m->elite_cost;
    a.cost_min = cost_min ? cost_min : m->cost_min;
    a.u_apply = u_apply;
    a.best = best;
    hipError_t e = cfk::launch_mppi_rollout(m->ks, a, h->stream);
    if (e == hipSuccess) e = cfk::launch_mppi_select(a, h->stream);
    return e == hipSuccess ? CF_OK : note(h, e);
}

cf_status cf_mppi_noise(cf_mppi* m, uint64_t iteration, float* eps) {
    if (!m) return CF_EINVAL;
    cf_handle* h = m->h;
    if (h->sticky != CF_OK) return h->sticky;
    const cfk::MppiArgs& b = m->base;
    if (check_dev(eps, (size_t)b.C * b.N * b.H * 4 * sizeof(float))) return CF_EINVAL;
    hipSetDevice(h->device);
    cfk::MppiArgs a = b;
    a.iter = iteration;
    a.eps_out = eps;
    hipError_t e = cfk::launch_mppi_noise(a, h->stream);
    return e == hipSuccess ? CF_OK : note(h, e);
}

}  // extern "C"
