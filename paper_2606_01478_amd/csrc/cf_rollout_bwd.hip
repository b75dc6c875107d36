// Adjoint rollout kernels: their launcher (the kernels and device code are in
// cf_rollout_impl.hpp, shared with the forward's translation unit).
#include "cf_rollout_impl.hpp"

namespace cfk {

hipError_t launch_rollout_bwd(const KernelSel& ks, const RollArgs& a, const int4* tiles, int n_tiles,
                              hipStream_t s) {
    CF_DISPATCH(launch_bwd_t, ks, a, tiles, n_tiles, s)
    return hipErrorInvalidValue;
}

}  // namespace cfk
