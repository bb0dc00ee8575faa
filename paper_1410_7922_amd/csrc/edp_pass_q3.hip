// Scan kernels of tiles 12, 13, 14, 15 for the truncated squared prior (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_SQ(12)
EDP_INSTANTIATE_TILE_SQ(13)
EDP_INSTANTIATE_TILE_SQ(14)
EDP_INSTANTIATE_TILE_SQ(15)

}  // namespace edp
