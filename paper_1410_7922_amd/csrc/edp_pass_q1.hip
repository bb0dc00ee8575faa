// Scan kernels of tiles 4, 5, 6, 7 with the general RMS (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_WIN(4)
EDP_INSTANTIATE_TILE_WIN(5)
EDP_INSTANTIATE_TILE_WIN(6)
EDP_INSTANTIATE_TILE_WIN(7)

}  // namespace edp
