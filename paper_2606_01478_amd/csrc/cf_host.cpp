// Host-only runtime pieces (no device calls); declarations in cf_host.hpp.
#include "cf_host.hpp"

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "cf_layout.hpp"

namespace cfh {

using namespace cfk;

cf_status validate_desc(const cf_desc* d, std::vector<int32_t>& counts, std::vector<uint8_t>& models,
                        std::vector<int32_t>& gidx, int64_t* D_out) {
    if (!d || !D_out) return CF_EINVAL;
    if (d->n_worlds < 1) return CF_EINVAL;
    const int M = d->n_worlds;
    counts.assign(M, 0);
    models.assign(M, 0);
    int64_t D = 0;
    for (int w = 0; w < M; ++w) {
        const int n = d->drones_per_world ? d->drones_per_world[w] : d->n_drones;
        if (n < 0) return CF_EINVAL;
        counts[w] = n;
        D += n;
        if (D > 2147483647LL) return CF_EINVAL;
        const int m = d->model_per_world ? d->model_per_world[w] : d->model;
        if (m != CF_MODEL_FP && m != CF_MODEL_ID) return CF_EINVAL;
        models[w] = (uint8_t)m;
    }
    if (d->control != CF_CTRL_ROTOR && d->control != CF_CTRL_ATT_PID && d->control != CF_CTRL_TORQUE &&
        d->control != CF_CTRL_POSITION)
        return CF_EINVAL;
    if (d->integrator != CF_INTEG_EULER && d->integrator != CF_INTEG_RK4) return CF_EINVAL;
    if (!(std::isfinite(d->dt) && d->dt > 0.f)) return CF_EINVAL;
    if (d->renorm_q != 0 && d->renorm_q != 1) return CF_EINVAL;
    if (d->ctrl_every < 0 || d->ctrl_every > CF_MAX_CTRL_EVERY) return CF_EINVAL;
    if (!d->params) return CF_EINVAL;
    if (d->n_gains < 0) return CF_EINVAL;
    gidx.assign(M, 0);
    if (d->gain_index) {
        for (int w = 0; w < M; ++w) {
            if (d->gain_index[w] < 0 || d->gain_index[w] >= std::max(d->n_gains, 1)) return CF_EINVAL;
            gidx[w] = d->gain_index[w];
        }
    }
    for (int w = 0; w < M; ++w) {
        const float* r = d->params + (size_t)w * CF_NPARAM;
        for (int i = 0; i < CF_NPARAM; ++i)
            if (!std::isfinite(r[i])) return CF_EINVAL;
        if (!(r[CF_P_MASS] > 0.f)) return CF_EINVAL;
        if (models[w] == CF_MODEL_FP) {
            for (int i = 0; i < 3; ++i)
                if (!(r[CF_P_J + i] > 0.f)) return CF_EINVAL;
            if (d->control != CF_CTRL_ROTOR && !(r[CF_P_THRUST + 2] > 0.f)) return CF_EINVAL;
            if (r[CF_P_JP] < 0.f) return CF_EINVAL;
        } else {
            if (!(r[CF_P_CF] > 0.f) || r[CF_P_CTAU] < 0.f) return CF_EINVAL;
        }
    }
    *D_out = D;
    return CF_OK;
}

// Reciprocals and differences are formed in binary32 exactly as a kernel would;
// the reference-speed terms (the hover speed W_r on the thrust curve, thrust,
// drag torque and slopes there) in double from the binary32 W_r the kernels use
// to convert rotor speeds, rounded once.
bool torque_proportional(const float* r, double* kappa) {
    const double k0 = r[P_THRUST], k1 = r[P_THRUST + 1], k2 = r[P_THRUST + 2];
    const double t0 = r[P_TORQUE], t1 = r[P_TORQUE + 1], t2 = r[P_TORQUE + 2];
    const double kk[3] = {k0, k1, k2}, tt[3] = {t0, t1, t2};
    int j = 2;
    while (j >= 0 && kk[j] == 0.0) --j;
    if (j < 0) return false;
    const double kap = tt[j] / kk[j];
    for (int i = 0; i < 3; ++i) {
        const double d = tt[i] - kap * kk[i];
        if (!(std::fabs(d) <= 0x1p-20 * std::max(std::fabs(tt[i]), std::fabs(kap * kk[i])))) return false;
    }
    *kappa = kap;
    return std::isfinite(kap);
}

void derive_record(const float* r, float* out) {
    std::memcpy(out, r, NPARAM * sizeof(float));
    std::fill(out + NPARAM, out + NREC, 0.f);
    const float m = r[P_MASS];
    out[D_INV_M] = 1.0f / m;
    for (int i = 0; i < 3; ++i) out[D_IJ + i] = 1.0f / r[P_J + i];
    out[D_DJ] = r[P_J + 2] - r[P_J + 1];
    out[D_DJ + 1] = r[P_J] - r[P_J + 2];
    out[D_DJ + 2] = r[P_J + 1] - r[P_J];
    out[D_INV_2K2] = 0.5f / r[P_THRUST + 2];
    for (int i = 0; i < 4; ++i) {
        const float tz = r[P_MIX_YAW + i];
        out[D_SG + i] = tz > 0.f ? -1.f : (tz < 0.f ? 1.f : 0.f);
    }
    const double k0 = r[P_THRUST], k1 = r[P_THRUST + 1], k2 = r[P_THRUST + 2];
    const double t0 = r[P_TORQUE], t1 = r[P_TORQUE + 1], t2 = r[P_TORQUE + 2];
    float wr = 0.f;
    if (k2 > 0.0) {
        // hover (m g / 4 per rotor) on the rising branch, else the vertex; never negative
        const double dh = k1 * k1 - 4.0 * k2 * (k0 - 0.25 * (double)m * r[P_GRAVITY]);
        const double w = ((dh > 0.0 ? std::sqrt(dh) : 0.0) - k1) / (2.0 * k2);
        wr = std::isfinite(w) ? (float)std::max(w, 0.0) : 0.f;
    }
    const double W = wr;
    const float k1w = wr > 0.f ? (float)std::max(k1 + 2.0 * k2 * W, 0.0) : (float)k1;
    const double fr = k0 + W * (k1 + k2 * W);
    const double tr = t0 + W * (t1 + t2 * W);
    double stx = 0.0, sty = 0.0, stz = 0.0, ssg = 0.0;
    for (int i = 0; i < 4; ++i) {
        stx += r[P_MIX_TX + i];
        sty += r[P_MIX_TY + i];
        stz += r[P_MIX_YAW + i];
        ssg += out[D_SG + i];
    }
    out[D_WR] = wr;
    out[D_W2] = 2.f * wr;
    out[D_K1W] = k1w;
    out[D_T1W] = (float)(t1 + 2.0 * t2 * W);
    out[D_FR] = (float)fr;
    out[D_F4R] = (float)(4.0 * fr);
    out[D_TXR] = (float)(fr * stx);
    out[D_TYR] = (float)(fr * sty);
    out[D_TZR] = (float)(tr * stz);
    out[D_SGR] = (float)(W * ssg);
    out[D_DISC_R] = (float)((double)k1w * k1w);
    out[D_VTX] = k2 > 0.0 ? (float)(-(double)k1w / (2.0 * k2)) : 0.f;
    const float cf = r[P_CF];
    out[D_CF_M] = cf / m;
    out[D_F_HOVER] = m * r[P_GRAVITY] / cf;
    double kap = 0.0;
    if (torque_proportional(r, &kap)) {
        out[D_TPROP] = 1.f;
        for (int i = 0; i < 4; ++i) out[D_TZK + i] = (float)(kap * r[P_MIX_YAW + i]);
    }
}

namespace {
int model_cost(int model, int ctrl) {
    if (model == MODEL_ID) return 2;
    return ctrl == CTRL_ROTOR ? 4 : 5;
}
}  // namespace

std::vector<Tile> tile_list(const std::vector<int32_t>& counts, const std::vector<int64_t>& offsets,
                            const std::vector<uint8_t>& models, int control, int tile, int* n_fp) {
    struct T {
        Tile v;
        int cost;
    };
    std::vector<T> ts;
    const int M = (int)counts.size();
    for (int w = 0; w < M; ++w) {
        const int n = counts[w];
        for (int s = 0; s < n; s += tile) {
            const int c = std::min(tile, n - s);
            const int waves = (c + 63) / 64;
            ts.push_back({{w, (int)(offsets[w] + s), c, (int)models[w]}, waves * model_cost(models[w], control)});
        }
    }
    std::stable_sort(ts.begin(), ts.end(), [](const T& a, const T& b) {
        if (a.v.model != b.v.model) return a.v.model < b.v.model;
        return a.cost > b.cost;
    });
    std::vector<Tile> v(ts.size());
    int nfp = 0;
    for (size_t i = 0; i < ts.size(); ++i) {
        v[i] = ts[i].v;
        nfp += (ts[i].v.model == MODEL_FP);
    }
    if (n_fp) *n_fp = nfp;
    return v;
}

std::vector<PackedTile> packed_tiles(const std::vector<int32_t>& counts, const std::vector<int64_t>& offsets,
                                     const std::vector<uint8_t>& models, int tile, std::vector<int32_t>* list,
                                     int* n_fp) {
    std::vector<PackedTile> v;
    list->clear();
    int nfp = 0;
    const int M = (int)counts.size();
    for (int model : {(int)MODEL_FP, (int)MODEL_ID}) {
        const int start = (int)list->size();
        for (int w = 0; w < M; ++w) {
            if (models[w] != model) continue;
            for (int i = 0; i < counts[w]; ++i) list->push_back((int32_t)(offsets[w] + i));
        }
        const int n = (int)list->size() - start;
        for (int s = 0; s < n; s += tile) {
            v.push_back({start + s, std::min(tile, n - s), model});
            nfp += (model == MODEL_FP);
        }
    }
    if (n_fp) *n_fp = nfp;
    return v;
}

bool cache_lookup(const std::string& path, const std::string& key, LaunchChoice* c) {
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    bool found = false;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char k[256];
        LaunchChoice x;
        if (std::sscanf(line, "%255s %d %d %d %d %f", k, &x.wq, &x.tile, &x.chunk, &x.split, &x.ms) != 6) continue;
        if (key == k) {
            *c = x;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

bool cache_store(const std::string& path, const std::string& key, const LaunchChoice& c) {
    std::vector<std::string> lines;
    if (FILE* f = std::fopen(path.c_str(), "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, f)) {
            char k[256];
            if (std::sscanf(line, "%255s", k) == 1 && key != k) {
                std::string l(line);
                if (l.empty() || l.back() != '\n') l += '\n';
                lines.push_back(l);
            }
        }
        std::fclose(f);
    }
    // create missing parent directories, outermost first
    for (size_t i = path.find('/', 1); i != std::string::npos; i = path.find('/', i + 1))
        mkdir(path.substr(0, i).c_str(), 0755);
    FILE* f = std::fopen(path.c_str(), "w");
    if (!f) return false;
    for (auto& l : lines) std::fputs(l.c_str(), f);
    std::fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), c.wq, c.tile, c.chunk, c.split, c.ms);
    std::fclose(f);
    return true;
}

int64_t ckpt_ubuf_offset(int T, int K, int S, int64_t D) {
    const int64_t nseg = ((int64_t)T + K - 1) / K;
    return nseg * S * D;
}

int64_t ckpt_tag_offset(int T, int K, int S, int64_t D, int kind) {
    int64_t n = ckpt_ubuf_offset(T, K, S, D);
    if (kind == CF_OBJ_BPTT_REWARD) n += (int64_t)T * 4 * D;
    return n;
}

int64_t ckpt_floats(int T, int K, int S, int64_t D, int kind) {
    return ckpt_tag_offset(T, K, S, D, kind) + CF_CKPT_TAG_FLOATS;
}

namespace {
struct Fnv {
    uint32_t h = 2166136261u;
    void bytes(const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 16777619u;
        }
    }
    template <class T>
    void add(const T& v) {
        bytes(&v, sizeof v);
    }
};
}  // namespace

uint32_t objective_hash(const cf_objective* obj) {
    Fnv f;
    const int32_t present = obj ? 1 : 0;
    f.add(present);
    if (!obj) return f.h;
    const int32_t flags =
        (obj->gain ? 1 : 0) | (obj->ref_table ? 2 : 0) | (obj->ref_offset ? 4 : 0) | (obj->ref_time_shift ? 8 : 0);
    f.add(obj->kind);
    f.add(flags);
    f.add(obj->ref_amp);
    f.add(obj->ref_period);
    f.add(obj->w_u);
    f.add(obj->policy_hidden);
    f.add(obj->ref_step0);
    for (int i = 0; i < 4; ++i) f.add(obj->policy_scale[i]);
    if (obj->kind == CF_OBJ_BPTT_REWARD) {
        f.add(obj->w_tilt);
        for (int i = 0; i < 4; ++i) f.add(obj->w_act[i]);
        for (int i = 0; i < 4; ++i) f.add(obj->w_dact[i]);
    }
    return f.h;
}

namespace {
uint32_t tag_checksum(const CkptTag& t) {
    Fnv f;
    f.bytes(t.w, sizeof(uint32_t) * (CF_CKPT_TAG_FLOATS - 1));
    return f.h;
}
}  // namespace

CkptTag make_tag(uint32_t handle_id, uint32_t generation, int T, int K, int S, int64_t D, const cf_objective* obj) {
    CkptTag t;
    std::memset(&t, 0, sizeof t);
    t.w[0] = TAG_MAGIC;
    t.w[1] = handle_id;
    t.w[2] = generation;
    t.w[3] = (uint32_t)T;
    t.w[4] = (uint32_t)K;
    t.w[5] = (uint32_t)S;
    t.w[6] = (uint32_t)D;
    t.w[7] = obj ? (uint32_t)obj->kind : 0xffffffffu;
    t.w[8] = objective_hash(obj);
    t.w[CF_CKPT_TAG_FLOATS - 1] = tag_checksum(t);
    return t;
}

bool tag_well_formed(const CkptTag& t) {
    return t.w[0] == TAG_MAGIC && t.w[CF_CKPT_TAG_FLOATS - 1] == tag_checksum(t);
}

void CkptRegistry::record(const void* ckpt, const CkptTag& tag) {
    auto it = map_.find(ckpt);
    if (it == map_.end() && map_.size() >= cap_ && !map_.empty()) {
        auto oldest = map_.begin();
        for (auto j = map_.begin(); j != map_.end(); ++j)
            if (j->second.w[2] < oldest->second.w[2]) oldest = j;
        map_.erase(oldest);
    }
    map_[ckpt] = tag;
}

cf_status CkptRegistry::match(const void* ckpt, int T, int K, int S, int64_t D, const cf_objective* obj,
                              CkptTag* out) const {
    auto it = map_.find(ckpt);
    if (it == map_.end()) return CF_ESTATE;
    const CkptTag& t = it->second;
    if (t.w[3] != (uint32_t)T || t.w[4] != (uint32_t)K || t.w[5] != (uint32_t)S || t.w[6] != (uint32_t)D)
        return CF_ESTATE;
    if (t.w[7] != (obj ? (uint32_t)obj->kind : 0xffffffffu) || t.w[8] != objective_hash(obj)) return CF_ESTATE;
    if (out) *out = t;
    return CF_OK;
}

}  // namespace cfh
