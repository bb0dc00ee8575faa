// Min-marginal scanline DP kernels of tiles 0, 1, 2, 3, 4, 5, 6, 7, 8 (dispatched from edp_dpm.hip).
#include "edp_dpm_kernel.hpp"

namespace edp {

EDP_DPM_TILE(0, 16, 1, 1, 1)
EDP_DPM_TILE(1, 32, 1, 1, 1)
EDP_DPM_TILE(2, 64, 1, 1, 1)
EDP_DPM_TILE(3, 16, 2, 1, 1)
EDP_DPM_TILE(4, 8, 4, 1, 1)
EDP_DPM_TILE(5, 16, 4, 1, 1)
EDP_DPM_TILE(6, 32, 2, 1, 1)
EDP_DPM_TILE(7, 64, 4, 1, 1)
EDP_DPM_TILE(8, 32, 8, 1, 1)

}  // namespace edp
