// Scan kernels of tiles 12, 13, 14, 15 for the truncated squared prior (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_QUAD(12)
EDP_INSTANTIATE_TILE_QUAD(13)
EDP_INSTANTIATE_TILE_QUAD(14)
EDP_INSTANTIATE_TILE_QUAD(15)

}  // namespace edp
