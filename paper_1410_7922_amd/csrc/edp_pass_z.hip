// Scan and marginal kernels of the three-dimensional label-space tiles 19, 20, 21 with every
// minimum search (instantiated here, dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE(19)
EDP_INSTANTIATE_TILE(20)
EDP_INSTANTIATE_TILE(21)
EDP_INSTANTIATE_TILE_WIN(19)
EDP_INSTANTIATE_TILE_WIN(20)
EDP_INSTANTIATE_TILE_WIN(21)

}  // namespace edp
