// Scan and marginal kernels of tiles 4, 5, 6, 7 (instantiated here, dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE(4)
EDP_INSTANTIATE_TILE(5)
EDP_INSTANTIATE_TILE(6)
EDP_INSTANTIATE_TILE(7)

}  // namespace edp
