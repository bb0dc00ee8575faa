// Scan kernels of tiles 8, 9, 10, 11 with the general RMS (instantiated here,
// dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE_WIN(8)
EDP_INSTANTIATE_TILE_WIN(9)
EDP_INSTANTIATE_TILE_WIN(10)
EDP_INSTANTIATE_TILE_WIN(11)

}  // namespace edp
