// Min-marginal scanline DP kernels of tiles 13, 14, 15 (dispatched from edp_dpm.hip).
#include "edp_dpm_kernel.hpp"

namespace edp {

EDP_DPM_TILE(13, 8, 1, 8, 1)
EDP_DPM_TILE(14, 4, 2, 4, 2)
EDP_DPM_TILE(15, 4, 8, 16, 2)

}  // namespace edp
