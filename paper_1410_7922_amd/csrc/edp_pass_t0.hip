// Scan and marginal kernels of tiles 0, 1, 2, 3 (instantiated here, dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE(0)
EDP_INSTANTIATE_TILE(1)
EDP_INSTANTIATE_TILE(2)
EDP_INSTANTIATE_TILE(3)

}  // namespace edp
