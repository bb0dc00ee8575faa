// Scan kernels of tiles 0, 1, 2, 3 for the truncated squared prior (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_SQ(0)
EDP_INSTANTIATE_TILE_SQ(1)
EDP_INSTANTIATE_TILE_SQ(2)
EDP_INSTANTIATE_TILE_SQ(3)

}  // namespace edp
