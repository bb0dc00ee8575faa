// Host dispatch of the EDP scan and marginal kernels: picks the tile's entry points,
// which live in the edp_pass_t*.hip translation units (edp_pass_kernel.hpp holds the
// kernels).
#include "edp_internal.hpp"

namespace edp {

template <int ID, int MS>
hipError_t pass_tile(int kind, int split, const PassArgs& a, int grid, int waves, hipStream_t s);
template <int ID, int MS> int occupancy_tile(int kind, int split, int waves, size_t lds);
template <int ID> hipError_t aggregate_tile(int dtype, const AggArgs& a, int grid, hipStream_t s);
hipError_t pass_win(const PassArgs& a, int grid, int waves, int ms, hipStream_t s);
int occupancy_win(int waves, int ms, size_t lds_bytes);
hipError_t aggregate_win(const AggArgs& a, int grid, hipStream_t s);

// counters, ticket word, trash slot, then one ring per compute wavefront plus the helper's
size_t pass_lds_bytes(int qt, int waves, int ring) {
    return (size_t)(2 * (MAX_WAVES + 1) + 4 + qt) * 4 + (size_t)(waves + 1) * ring * qt * 4;
}

hipError_t launch_edp_pass(int tile, int dtype, int split, int ms, const PassArgs& a, int grid, int waves,
                           hipStream_t s) {
    if (waves < 1 || waves > MAX_WAVES) return hipErrorInvalidValue;
    if (dtype == KIND_WINDOW)
        return tile == WIN_TILE && split == 1 && (ms == MS_LINEAR || ms == MS_WINDOW) ? pass_win(a, grid, waves, ms, s)
                                                                                     : hipErrorInvalidValue;
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                                                   \
    case id:                                                                                           \
        return ms == MS_WALK      ? pass_tile<id, MS_WALK>(dtype, split, a, grid, waves, s)       \
               : ms == MS_WINDOW1 ? pass_tile<id, MS_WINDOW1>(dtype, split, a, grid, waves, s)    \
               : ms == MS_WINDOW  ? pass_tile<id, MS_WINDOW>(dtype, split, a, grid, waves, s)      \
                                   : pass_tile<id, MS_LINEAR>(dtype, split, a, grid, waves, s);
        EDP_TILE_LIST(EDP_CASE)
#define EDP_CASE3(id, px, kx, py, ky, kz) EDP_CASE(id, px, kx, py, ky)
        EDP_TILE3_LIST(EDP_CASE3)
#undef EDP_CASE3
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_edp_aggregate_win(const AggArgs& a, int grid, hipStream_t s) { return aggregate_win(a, grid, s); }

hipError_t launch_edp_aggregate(int tile, int dtype, const AggArgs& a, int grid, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky) \
    case id:                         \
        return aggregate_tile<id>(dtype, a, grid, s);
        EDP_TILE_LIST(EDP_CASE)
#define EDP_CASE3(id, px, kx, py, ky, kz) EDP_CASE(id, px, kx, py, ky)
        EDP_TILE3_LIST(EDP_CASE3)
#undef EDP_CASE3
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

int pass_capacity(int tile, int dtype, int split, int ms, int waves, size_t lds_bytes) {
    int per_cu = 1;
    if (dtype == KIND_WINDOW) {
        per_cu = occupancy_win(waves, ms, lds_bytes);
        tile = -1;
    }
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                                                \
    case id:                                                                                        \
        per_cu = ms == MS_WALK      ? occupancy_tile<id, MS_WALK>(dtype, split, waves, lds_bytes)    \
                 : ms == MS_WINDOW1 ? occupancy_tile<id, MS_WINDOW1>(dtype, split, waves, lds_bytes) \
                 : ms == MS_WINDOW  ? occupancy_tile<id, MS_WINDOW>(dtype, split, waves, lds_bytes)   \
                                     : occupancy_tile<id, MS_LINEAR>(dtype, split, waves, lds_bytes);  \
        break;
        EDP_TILE_LIST(EDP_CASE)
#define EDP_CASE3(id, px, kx, py, ky, kz) EDP_CASE(id, px, kx, py, ky)
        EDP_TILE3_LIST(EDP_CASE3)
#undef EDP_CASE3
#undef EDP_CASE
    }
    int dev = 0, cus = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1;
    return per_cu * cus;
}

}  // namespace edp
