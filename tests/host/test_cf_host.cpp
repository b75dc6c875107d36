// CPU tests of the host-only runtime (paper_2606_01478_amd/csrc/cf_host.cpp):
// descriptor validation, derived records, tile lists, the autotune cache file
// and the checkpoint tags. Built with AddressSanitizer and UBSan by
// tests/test_host_sanitized.py; exits non-zero on the first failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2606_01478_amd/csrc/cf_host.hpp"
#include "../../paper_2606_01478_amd/csrc/cf_layout.hpp"

static int g_checks = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        ++g_checks;                                                              \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

// a valid two-world descriptor (first-principles + identified) over owned arrays
struct DescFixture {
    std::vector<int32_t> counts{3, 5};
    std::vector<uint8_t> models{CF_MODEL_FP, CF_MODEL_ID};
    std::vector<float> params;
    std::vector<int32_t> gidx{0, 1};
    cf_desc d;
    DescFixture() {
        params.assign(2 * CF_NPARAM, 0.f);
        float* r = params.data();
        r[CF_P_MASS] = 0.027f; r[CF_P_GRAVITY] = 9.81f;
        r[CF_P_J] = 1.4e-5f; r[CF_P_J + 1] = 1.4e-5f; r[CF_P_J + 2] = 2.2e-5f;
        r[CF_P_THRUST + 2] = 3e-10f; r[CF_P_TORQUE + 2] = 1.8e-12f;
        const float mix_yaw[4] = {-1.f, 1.f, -1.f, 1.f};
        for (int i = 0; i < 4; ++i) r[CF_P_MIX_YAW + i] = mix_yaw[i];
        float* q = params.data() + CF_NPARAM;
        q[CF_P_MASS] = 0.03f; q[CF_P_GRAVITY] = 9.81f; q[CF_P_CF] = 1.f; q[CF_P_CTAU] = 33.f;
        std::memset(&d, 0, sizeof d);
        d.n_worlds = 2;
        d.drones_per_world = counts.data();
        d.model_per_world = models.data();
        d.control = CF_CTRL_ATT_PID;
        d.integrator = CF_INTEG_RK4;
        d.dt = 0.002f;
        d.renorm_q = 1;
        d.params = params.data();
        d.n_gains = 2;
        d.gain_index = gidx.data();
        d.device = -1;
    }
    cf_status run() {
        std::vector<int32_t> c, g;
        std::vector<uint8_t> m;
        int64_t D = -1;
        return cfh::validate_desc(&d, c, m, g, &D);
    }
};

static void test_validate_desc() {
    {
        DescFixture f;
        std::vector<int32_t> c, g;
        std::vector<uint8_t> m;
        int64_t D = -1;
        CHECK(cfh::validate_desc(&f.d, c, m, g, &D) == CF_OK);
        CHECK(D == 8 && c[1] == 5 && m[1] == CF_MODEL_ID && g[1] == 1);
    }
    {
        std::vector<int32_t> c, g;
        std::vector<uint8_t> m;
        int64_t D = 0;
        CHECK(cfh::validate_desc(nullptr, c, m, g, &D) == CF_EINVAL);
        DescFixture f;
        CHECK(cfh::validate_desc(&f.d, c, m, g, nullptr) == CF_EINVAL);
    }
    auto bad = [](void (*edit)(DescFixture&)) {
        DescFixture f;
        edit(f);
        return f.run() == CF_EINVAL;
    };
    CHECK(bad([](DescFixture& f) { f.d.n_worlds = 0; }));
    CHECK(bad([](DescFixture& f) { f.counts[0] = -1; }));
    CHECK(bad([](DescFixture& f) { f.counts[0] = 2147483647; }));
    CHECK(bad([](DescFixture& f) { f.models[1] = 7; }));
    CHECK(bad([](DescFixture& f) { f.d.control = 9; }));
    CHECK(bad([](DescFixture& f) { f.d.integrator = 2; }));
    CHECK(bad([](DescFixture& f) { f.d.dt = 0.f; }));
    CHECK(bad([](DescFixture& f) { f.d.dt = NAN; }));
    CHECK(bad([](DescFixture& f) { f.d.renorm_q = 2; }));
    CHECK(bad([](DescFixture& f) { f.d.ctrl_every = -1; }));
    CHECK(bad([](DescFixture& f) { f.d.ctrl_every = CF_MAX_CTRL_EVERY + 1; }));
    CHECK(bad([](DescFixture& f) { f.d.params = nullptr; }));
    CHECK(bad([](DescFixture& f) { f.d.n_gains = -1; }));
    CHECK(bad([](DescFixture& f) { f.gidx[1] = 2; }));
    CHECK(bad([](DescFixture& f) { f.params[5] = INFINITY; }));
    CHECK(bad([](DescFixture& f) { f.params[CF_P_MASS] = 0.f; }));
    CHECK(bad([](DescFixture& f) { f.params[CF_P_J + 2] = -1e-5f; }));
    CHECK(bad([](DescFixture& f) { f.params[CF_P_THRUST + 2] = 0.f; }));
    CHECK(bad([](DescFixture& f) { f.params[CF_P_JP] = -1e-9f; }));
    CHECK(bad([](DescFixture& f) { f.params[CF_NPARAM + CF_P_CF] = 0.f; }));
    CHECK(bad([](DescFixture& f) { f.params[CF_NPARAM + CF_P_CTAU] = -1.f; }));
    // the rotor interface needs no thrust curve for the controller
    DescFixture f;
    f.d.control = CF_CTRL_ROTOR;
    f.params[CF_P_THRUST + 2] = 0.f;
    CHECK(f.run() == CF_OK);
}

static void test_derive_record() {
    DescFixture f;
    float out[cfk::NREC];
    cfh::derive_record(f.params.data(), out);
    const double m = 0.027, g = 9.81, k2 = 3e-10;
    const double wr = out[cfk::D_WR];
    CHECK(std::fabs(k2 * wr * wr - m * g / 4) <= 1e-6 * m * g);
    CHECK(out[cfk::D_W2] == 2.f * out[cfk::D_WR]);
    CHECK(out[cfk::D_INV_M] == 1.0f / 0.027f);
    CHECK(out[cfk::D_IJ + 2] == 1.0f / 2.2e-5f);
    CHECK(out[cfk::D_DJ] == 2.2e-5f - 1.4e-5f);   // Jz - Jy
    CHECK(out[cfk::D_SG] == 1.f && out[cfk::D_SG + 1] == -1.f);   // spin = -sign(yaw mixing)
    CHECK(std::fabs(out[cfk::D_F4R] - m * g) <= 1e-6);              // four rotors hover
    for (int i = 0; i < CF_NPARAM; ++i) CHECK(out[i] == f.params[i]);
    float outi[cfk::NREC];
    cfh::derive_record(f.params.data() + CF_NPARAM, outi);
    CHECK(std::fabs(outi[cfk::D_F_HOVER] - 0.03f * 9.81f) <= 1e-6f);
    CHECK(outi[cfk::D_CF_M] == 1.f / 0.03f);
    // drag torque proportional to thrust: flagged, yaw coefficients scaled by kappa
    std::vector<float> r(f.params.begin(), f.params.begin() + CF_NPARAM);
    for (int j = 0; j < 3; ++j) r[CF_P_TORQUE + j] = 0.006f * r[CF_P_THRUST + j];
    double kap = 0.0;
    CHECK(cfh::torque_proportional(r.data(), &kap));
    CHECK(std::fabs(kap - 0.006) <= 1e-9);
    cfh::derive_record(r.data(), out);
    CHECK(out[cfk::D_TPROP] == 1.f);
    for (int i = 0; i < 4; ++i) CHECK(out[cfk::D_TZK + i] == (float)(kap * r[CF_P_MIX_YAW + i]));
    // a linear term in the torque only: not proportional
    r[CF_P_TORQUE + 1] = 1e-9f;
    CHECK(!cfh::torque_proportional(r.data(), &kap));
    cfh::derive_record(r.data(), out);
    CHECK(out[cfk::D_TPROP] == 0.f);
    // no thrust curve at all: not proportional
    for (int j = 0; j < 3; ++j) r[CF_P_THRUST + j] = 0.f;
    CHECK(!cfh::torque_proportional(r.data(), &kap));
}

static void test_packed_tiles() {
    std::vector<int32_t> counts{130, 0, 1, 64, 200, 7, 3};
    std::vector<uint8_t> models{1, 0, 0, 1, 0, 1, 0};
    std::vector<int64_t> off{0};
    for (int c : counts) off.push_back(off.back() + c);
    std::vector<int32_t> world_of(off.back());
    for (size_t w = 0; w < counts.size(); ++w)
        for (int64_t d = off[w]; d < off[w + 1]; ++d) world_of[d] = (int32_t)w;
    for (int tile : {64, 128, 256}) {
        int nfp = -1;
        std::vector<int32_t> list;
        auto v = cfh::packed_tiles(counts, off, models, tile, &list, &nfp);
        CHECK((int64_t)list.size() == off.back());
        std::vector<int> seen(off.back(), 0);
        for (int32_t d : list) seen[d]++;
        for (int s : seen) CHECK(s == 1);
        // first-principles drones first, each model's drones world after world, in order
        for (size_t i = 1; i < list.size(); ++i) {
            const int m0 = models[world_of[list[i - 1]]], m1 = models[world_of[list[i]]];
            CHECK(m0 <= m1);
            if (m0 == m1) CHECK(list[i] > list[i - 1]);
        }
        int covered = 0, fp_tiles = 0;
        for (size_t k = 0; k < v.size(); ++k) {
            const auto& t = v[k];
            CHECK(t.first == covered);
            CHECK(t.count >= 1 && t.count <= tile);
            for (int i = 0; i < t.count; ++i) CHECK(models[world_of[list[t.first + i]]] == t.model);
            // full tiles except the last of each model
            const bool last_of_model = k + 1 == v.size() || v[k + 1].model != t.model;
            if (!last_of_model) CHECK(t.count == tile);
            fp_tiles += t.model == 0;
            covered += t.count;
        }
        CHECK(covered == (int)off.back());
        CHECK(fp_tiles == nfp);
    }
}

static void test_tile_list() {
    std::vector<int32_t> counts{130, 0, 1, 64, 200, 7};
    std::vector<uint8_t> models{1, 0, 0, 1, 0, 1};
    std::vector<int64_t> off{0};
    for (int c : counts) off.push_back(off.back() + c);
    for (int tile : {64, 128, 256}) {
        int nfp = -1;
        auto v = cfh::tile_list(counts, off, models, CF_CTRL_ATT_PID, tile, &nfp);
        std::vector<int> seen(off.back(), 0);
        int fp_seen = 0;
        bool id_started = false;
        int prev_cost = 1 << 30;
        int prev_model = -1;
        for (const auto& t : v) {
            CHECK(t.count >= 1 && t.count <= tile);
            CHECK(t.model == models[t.world]);
            CHECK(t.first >= off[t.world] && t.first + t.count <= off[t.world + 1]);
            for (int k = 0; k < t.count; ++k) seen[t.first + k]++;
            if (t.model == 0) {
                CHECK(!id_started);
                ++fp_seen;
            } else {
                id_started = true;
            }
            const int cost = ((t.count + 63) / 64) * (t.model == 1 ? 2 : 5);
            if (t.model == prev_model) CHECK(cost <= prev_cost);
            prev_cost = cost;
            prev_model = t.model;
        }
        for (int s : seen) CHECK(s == 1);
        CHECK(fp_seen == nfp);
    }
}

static void test_cache(const std::string& dir) {
    const std::string path = dir + "/sub/cache.txt";
    cfh::LaunchChoice c;
    CHECK(!cfh::cache_lookup(path, "k1", &c));
    cfh::LaunchChoice a;
    a.wq = 1; a.tile = 128; a.chunk = 100; a.split = 0; a.ms = 2.5f;
    CHECK(cfh::cache_store(path, "k1", a));
    a.tile = 256;
    CHECK(cfh::cache_store(path, "k2", a));
    a.tile = 64; a.chunk = 25;
    CHECK(cfh::cache_store(path, "k1", a));   // replaces k1
    {
        FILE* f = std::fopen(path.c_str(), "a");
        std::fputs("garbage line without numbers\nk3 1 2\n", f);
        std::fclose(f);
    }
    CHECK(cfh::cache_lookup(path, "k1", &c) && c.tile == 64 && c.chunk == 25 && c.wq == 1 && c.split == 0);
    CHECK(cfh::cache_lookup(path, "k2", &c) && c.tile == 256);
    CHECK(!cfh::cache_lookup(path, "k3", &c));
    int lines = 0;
    FILE* f = std::fopen(path.c_str(), "r");
    char buf[512];
    while (std::fgets(buf, sizeof buf, f)) lines += std::strncmp(buf, "k1 ", 3) == 0;
    std::fclose(f);
    CHECK(lines == 1);
}

static void test_tags() {
    cf_objective o;
    std::memset(&o, 0, sizeof o);
    o.ref_amp = 1.f; o.ref_period = 4.f; o.w_u = 1e-3f;
    float g = 0.f;
    cf_objective og = o;
    og.gain = &g;
    cf_objective orw = o;
    orw.kind = CF_OBJ_BPTT_REWARD;
    CHECK(cfh::objective_hash(&o) != cfh::objective_hash(&og));
    CHECK(cfh::objective_hash(&o) != cfh::objective_hash(&orw));
    CHECK(cfh::objective_hash(&o) != cfh::objective_hash(nullptr));
    cf_objective o2 = o;
    o2.w_u = 2e-3f;
    CHECK(cfh::objective_hash(&o) != cfh::objective_hash(&o2));
    cf_objective r2 = orw;
    r2.w_dact[3] = 0.5f;
    CHECK(cfh::objective_hash(&orw) != cfh::objective_hash(&r2));

    const cfh::CkptTag t = cfh::make_tag(7, 3, 500, 25, 13, 1024, &og);
    CHECK(cfh::tag_well_formed(t));
    for (int i = 0; i < CF_CKPT_TAG_FLOATS; ++i) {
        cfh::CkptTag u = t;
        u.w[i] ^= 0x10u;
        CHECK(!cfh::tag_well_formed(u));
    }
    CHECK(cfh::ckpt_floats(500, 25, 13, 1024, CF_OBJ_TRACKING) == 20LL * 13 * 1024 + CF_CKPT_TAG_FLOATS);
    CHECK(cfh::ckpt_floats(501, 25, 13, 1024, CF_OBJ_TRACKING) == 21LL * 13 * 1024 + CF_CKPT_TAG_FLOATS);
    CHECK(cfh::ckpt_floats(40, 10, 25, 16, CF_OBJ_BPTT_REWARD) == 4LL * 25 * 16 + 40LL * 4 * 16 + CF_CKPT_TAG_FLOATS);
    CHECK(cfh::ckpt_ubuf_offset(40, 10, 25, 16) == 4LL * 25 * 16);
    CHECK(cfh::ckpt_tag_offset(40, 10, 25, 16, CF_OBJ_BPTT_REWARD) == 4LL * 25 * 16 + 40LL * 4 * 16);

    // two forwards before their backwards; re-use of a buffer; mismatches
    cfh::CkptRegistry reg(4);
    int bufA, bufB;
    reg.record(&bufA, cfh::make_tag(7, 1, 500, 25, 13, 1024, &og));
    reg.record(&bufB, cfh::make_tag(7, 2, 500, 50, 13, 1024, &og));
    cfh::CkptTag got;
    CHECK(reg.match(&bufA, 500, 25, 13, 1024, &og, &got) == CF_OK && got.w[2] == 1);
    CHECK(reg.match(&bufB, 500, 50, 13, 1024, &og, &got) == CF_OK && got.w[2] == 2);
    CHECK(reg.match(&bufA, 500, 50, 13, 1024, &og, &got) == CF_ESTATE);   // other K
    CHECK(reg.match(&bufA, 499, 25, 13, 1024, &og, &got) == CF_ESTATE);   // other T
    CHECK(reg.match(&bufA, 500, 25, 25, 1024, &og, &got) == CF_ESTATE);   // other S
    CHECK(reg.match(&bufA, 500, 25, 13, 1023, &og, &got) == CF_ESTATE);   // other D
    CHECK(reg.match(&bufA, 500, 25, 13, 1024, &o, &got) == CF_ESTATE);    // gain dropped
    CHECK(reg.match(&bufA, 500, 25, 13, 1024, &orw, &got) == CF_ESTATE);  // other kind
    CHECK(reg.match(&bufA, 500, 25, 13, 1024, nullptr, &got) == CF_ESTATE);
    int never;
    CHECK(reg.match(&never, 500, 25, 13, 1024, &og, &got) == CF_ESTATE);
    reg.record(&bufA, cfh::make_tag(7, 3, 100, 10, 13, 1024, &o));        // buffer re-used
    CHECK(reg.match(&bufA, 500, 25, 13, 1024, &og, &got) == CF_ESTATE);
    CHECK(reg.match(&bufA, 100, 10, 13, 1024, &o, &got) == CF_OK && got.w[2] == 3);
    // bounded: the oldest generation goes first
    int more[3];
    for (int i = 0; i < 3; ++i) reg.record(&more[i], cfh::make_tag(7, 4 + i, 10, 1, 13, 8, &o));
    CHECK(reg.size() == 4);
    CHECK(reg.match(&bufB, 500, 50, 13, 1024, &og, &got) == CF_ESTATE);   // generation 2 dropped
    CHECK(reg.match(&bufA, 100, 10, 13, 1024, &o, &got) == CF_OK);
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : "/tmp";
    test_validate_desc();
    test_derive_record();
    test_tile_list();
    test_packed_tiles();
    test_cache(dir);
    test_tags();
    std::printf("host tests passed: %d checks\n", g_checks);
    return 0;
}
