// Scan and marginal kernels of tiles 8, 9, 10, 11 (instantiated here, dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE(8)
EDP_INSTANTIATE_TILE(9)
EDP_INSTANTIATE_TILE(10)
EDP_INSTANTIATE_TILE(11)

}  // namespace edp
