// Scan kernels of tiles 12, 13, 14, 15 with the general RMS (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_WIN(12)
EDP_INSTANTIATE_TILE_WIN(13)
EDP_INSTANTIATE_TILE_WIN(14)
EDP_INSTANTIATE_TILE_WIN(15)

}  // namespace edp
