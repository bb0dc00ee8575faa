// Host dispatch of the min-marginal scanline DP (kernels in edp_dpm_kernel.hpp, instantiated
// per tile in edp_dpm_a.hip, edp_dpm_b.hip and edp_dpm_c.hip).
#include "edp_internal.hpp"

namespace edp {

template <int ID>
hipError_t dpm_tile(int dtype, const DpmArgs& a, int grid, bool forward, hipStream_t s);

hipError_t launch_dp_marginals(int tile, int dtype, const DpmArgs& a, int grid, bool forward, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky) \
    case id:                         \
        return dpm_tile<id>(dtype, a, grid, forward, s);
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace edp
