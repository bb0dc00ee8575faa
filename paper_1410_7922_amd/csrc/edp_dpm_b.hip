// Min-marginal scanline DP kernels of tiles 9, 10, 11, 12 (dispatched from edp_dpm.hip).
#include "edp_dpm_kernel.hpp"

namespace edp {

EDP_DPM_TILE(9, 4, 4, 4, 4)
EDP_DPM_TILE(10, 4, 4, 16, 1)
EDP_DPM_TILE(11, 8, 2, 8, 2)
EDP_DPM_TILE(12, 8, 4, 8, 4)

}  // namespace edp
