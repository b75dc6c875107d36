// Host-only part of the runtime behind include/cfsim.h: everything that needs
// no device -- descriptor validation, the derived per-world records, the
// per-world tile lists of uneven batches, the autotune cache file, and the
// checkpoint tag that ties a backward call to the forward that filled its
// checkpoint buffer. Plain C++17 (no HIP): the library links it, and a CPU
// test builds it on its own under AddressSanitizer and UBSan.
#pragma once
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/cfsim.h"

namespace cfh {

// ---- descriptor and parameter records -------------------------------------------

// Validates *d; on success fills the per-world drone counts, models and gain
// indices and the total drone count. Returns CF_EINVAL on any violation of the
// cf_desc contract (header), CF_OK otherwise.
cf_status validate_desc(const cf_desc* d, std::vector<int32_t>& counts, std::vector<uint8_t>& models,
                        std::vector<int32_t>& gidx, int64_t* D_out);

// out[0..NREC): the public record r[0..CF_NPARAM) followed by the constants the
// kernels read instead of forming them (reciprocals, inertia differences, the
// reference-speed terms of the first-principles model, c_f / m and the hover
// thrust of the identified model).
void derive_record(const float* r, float* out);

// True when the rotor drag-torque polynomial is the thrust polynomial times one
// constant kappa (t_j = kappa k_j for j = 0, 1, 2, to 2^-20 relative); *kappa
// receives it. The reduced kernel variants then form the yaw torque from the
// thrust differences (coefficients kappa * yaw mixing, D_TZK).
bool torque_proportional(const float* r, double* kappa);

// ---- uneven batches --------------------------------------------------------------

struct Tile {
    int world, first, count, model;
};

// Per-world tiles of at most `tile` drones {world, first drone, count, model}:
// first-principles tiles first, within a model in longest-processing-time
// order (cost = 64-lane waves x model cost, ties by position). *n_fp receives
// the number of first-principles tiles.
std::vector<Tile> tile_list(const std::vector<int32_t>& counts, const std::vector<int64_t>& offsets,
                            const std::vector<uint8_t>& models, int control, int tile, int* n_fp);

// Packed tiles of the held-step kernels: the drones of each model listed world
// after world (first-principles worlds first, worlds in index order, a world's
// drones in order) in *list, cut into tiles of `tile` consecutive entries
// {first entry, count, model}, so that every tile but each model's last is full
// and a tile may span several worlds of its model. *n_fp receives the number of
// first-principles tiles (they come first).
struct PackedTile {
    int first, count, model;
};
std::vector<PackedTile> packed_tiles(const std::vector<int32_t>& counts, const std::vector<int64_t>& offsets,
                                     const std::vector<uint8_t>& models, int tile, std::vector<int32_t>* list,
                                     int* n_fp);

// ---- autotune cache ---------------------------------------------------------------

struct LaunchChoice {
    int wq = 0, tile = 64, chunk = 0, split = 1;
    float ms = 0.f;
};

// One line per handle signature: "<key> <wq> <tile> <chunk> <split> <ms>".
// Lookup keeps the last well-formed line of the key; malformed lines are
// skipped. Store rewrites the file with the key's line replaced.
bool cache_lookup(const std::string& path, const std::string& key, LaunchChoice* c);
bool cache_store(const std::string& path, const std::string& key, const LaunchChoice& c);

// ---- checkpoint buffers and their tag ---------------------------------------------

constexpr uint32_t TAG_MAGIC = 0x4b434643u;  // "CFCK"

struct CkptTag {
    uint32_t w[CF_CKPT_TAG_FLOATS];
};

// Floats of a checkpoint buffer for (T, K): ceil(T/K) states [S][D], then for
// the reward objective the applied commands [T][4][D], then the tag.
int64_t ckpt_floats(int T, int K, int S, int64_t D, int kind);
// Offset (floats) of the applied commands and of the tag inside that buffer.
int64_t ckpt_ubuf_offset(int T, int K, int S, int64_t D);
int64_t ckpt_tag_offset(int T, int K, int S, int64_t D, int kind);

// FNV-1a hash of what of the objective the backward must share with the
// forward: no objective / its kind, which optional inputs are present (gain,
// table, offsets) and its scalar weights.
uint32_t objective_hash(const cf_objective* obj);

// {magic, handle id, generation, T, K, S, D, kind, objective hash, 0.., checksum}
CkptTag make_tag(uint32_t handle_id, uint32_t generation, int T, int K, int S, int64_t D,
                 const cf_objective* obj);
bool tag_well_formed(const CkptTag& t);

// The tags of the forwards with a checkpoint buffer run on one handle, by
// buffer address (bounded; the oldest generation is dropped first). A backward
// is accepted only for a buffer whose latest forward on this handle had the
// same T, K, state size, drone count and objective; the tag returned is what
// the device then finds in the buffer unless it was overwritten since.
class CkptRegistry {
public:
    explicit CkptRegistry(size_t capacity = 256) : cap_(capacity) {}
    void record(const void* ckpt, const CkptTag& tag);
    cf_status match(const void* ckpt, int T, int K, int S, int64_t D, const cf_objective* obj,
                    CkptTag* out) const;
    size_t size() const { return map_.size(); }

private:
    size_t cap_;
    std::map<const void*, CkptTag> map_;
};

}  // namespace cfh
