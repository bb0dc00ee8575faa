// Scan kernels of tiles 4, 5, 6, 7 for the truncated squared prior (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_SQ(4)
EDP_INSTANTIATE_TILE_SQ(5)
EDP_INSTANTIATE_TILE_SQ(6)
EDP_INSTANTIATE_TILE_SQ(7)

}  // namespace edp
