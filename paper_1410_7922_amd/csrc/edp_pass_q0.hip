// Scan kernels of tiles 0, 1, 2, 3 with the general RMS (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_WIN(0)
EDP_INSTANTIATE_TILE_WIN(1)
EDP_INSTANTIATE_TILE_WIN(2)
EDP_INSTANTIATE_TILE_WIN(3)

}  // namespace edp
