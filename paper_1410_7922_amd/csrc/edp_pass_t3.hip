// Scan and marginal kernels of tiles 12, 13, 14, 15 (instantiated here, dispatched from edp_pass.hip).
#include "edp_pass_kernel.hpp"

namespace edp {

EDP_INSTANTIATE_TILE(12)
EDP_INSTANTIATE_TILE(13)
EDP_INSTANTIATE_TILE(14)
EDP_INSTANTIATE_TILE(15)

// label-window solve: 8 x 8 frames on the window tile; ms MS_WINDOW (T <= 3) or MS_LINEAR
template <int MS>
static hipError_t run_win(const PassArgs& a, int grid, int waves, hipStream_t s) {
    const size_t lds = pass_lds_bytes(WinTile::QT, waves, a.ring) + win_lds_bytes(waves);
    hipLaunchKernelGGL((edp_pass_kernel<WinTile, int32_t, 1, pass_pf<WinTile>(), true, MS>), dim3(grid),
                       dim3(64 * (waves + 2)), lds, s, a);
    return hipGetLastError();
}

hipError_t pass_win(const PassArgs& a, int grid, int waves, int ms, hipStream_t s) {
    return ms == MS_WINDOW ? run_win<MS_WINDOW>(a, grid, waves, s) : run_win<MS_LINEAR>(a, grid, waves, s);
}

template <int MS>
static int win_occupancy(int waves, size_t lds_bytes) {
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, edp_pass_kernel<WinTile, int32_t, 1, pass_pf<WinTile>(), true, MS>, 64 * (waves + 2),
            lds_bytes + win_lds_bytes(waves)) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu;
}

int occupancy_win(int waves, int ms, size_t lds_bytes) {
    return ms == MS_WINDOW ? win_occupancy<MS_WINDOW>(waves, lds_bytes) : win_occupancy<MS_LINEAR>(waves, lds_bytes);
}

hipError_t aggregate_win(const AggArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((edp_aggregate_kernel<WinTile, int32_t, true>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace edp
