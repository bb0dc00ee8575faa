// Scan kernels of tiles 8, 9, 10, 11 for the truncated squared prior (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_SQ(8)
EDP_INSTANTIATE_TILE_SQ(9)
EDP_INSTANTIATE_TILE_SQ(10)
EDP_INSTANTIATE_TILE_SQ(11)

}  // namespace edp
