// Scan and marginal kernels of the wide-vertex tiles (a vertex on several wavefronts),
// instantiated and dispatched here.
#include "edp_pass_mv.hpp"

namespace edp {

template <int ID> struct MvTileOf;
#define EDP_MV_OF(id, kx, ky, nv) \
    template <> struct MvTileOf<id> { using type = MvTile<kx, ky, nv>; };
EDP_MV_TILE_LIST(EDP_MV_OF)
#undef EDP_MV_OF
#define EDP_MV3_OF(id, kz, nv) \
    template <> struct MvTileOf<id> { using type = MvTile3<kz, nv>; };
EDP_MV3_TILE_LIST(EDP_MV3_OF)
#undef EDP_MV3_OF

// Prefetch depth in steps: the loads of a step are few, so several steps stay in flight (fewer
// where a lane holds more labels, or the helpers of eight slabs need more registers).
template <class M>
constexpr int mv_pf() { return M::E <= 4 && M::NV <= 4 ? 4 : 2; }

template <class M, class CK, int MS, bool NT = false>
static hipError_t run_mv(const PassArgs& a, int grid, int rows, hipStream_t s) {
    const size_t lds = mv_lds_bytes_t<M, MS == MS_WINDOW1 ? 1 : 2>(rows, a.ring);
    hipLaunchKernelGGL((edp_pass_mv_kernel<M, CK, MS, mv_pf<M>(), NT>), dim3(grid), dim3(64 * (M::NV * rows + 2)), lds,
                       s, a);
    return hipGetLastError();
}

template <class M, class CK, int MS>
static int occ_mv(int rows, size_t lds) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, edp_pass_mv_kernel<M, CK, MS, mv_pf<M>(), false>,
                                                     64 * (M::NV * rows + 2), lds) != hipSuccess)
        blocks = 1;
    return blocks < 1 ? 1 : blocks;
}

// cost kind: 1 int16 (element loads), 2 int32, 3 int16 in aligned pairs; nt: non-temporal sums
// (instantiated for int32 costs, the large motion volumes)
template <class M, int MS>
static hipError_t kind_mv(int kind, const PassArgs& a, int grid, int rows, hipStream_t s, bool nt) {
    if (kind == 1) return run_mv<M, int16_t, MS>(a, grid, rows, s);
    if (kind == 3) {
        if constexpr (M::KX % 2 == 0) return run_mv<M, Pair16, MS>(a, grid, rows, s);
        return hipErrorInvalidValue;
    }
    return nt ? run_mv<M, int32_t, MS, true>(a, grid, rows, s) : run_mv<M, int32_t, MS>(a, grid, rows, s);
}
template <class M, int MS>
static int kind_occ(int kind, int rows, size_t lds) {
    if (kind == 1) return occ_mv<M, int16_t, MS>(rows, lds);
    if (kind == 3) {
        if constexpr (M::KX % 2 == 0) return occ_mv<M, Pair16, MS>(rows, lds);
        return 1;
    }
    return occ_mv<M, int32_t, MS>(rows, lds);
}

hipError_t launch_edp_pass_mv(int tile, int kind, int ms, const PassArgs& a, int grid, int rows, hipStream_t s,
                              bool nt) {
    if (ms != MS_WINDOW && ms != MS_WINDOW1) return hipErrorInvalidValue;
    switch (tile) {
#define EDP_CASE(id, kx, ky, nv)                                                                          \
    case id:                                                                                              \
        if (rows < 1 || rows * nv > MV_MAX_WAVES) return hipErrorInvalidValue;                            \
        return ms == MS_WINDOW1 ? kind_mv<MvTileOf<id>::type, MS_WINDOW1>(kind, a, grid, rows, s, nt)      \
                                : kind_mv<MvTileOf<id>::type, MS_WINDOW>(kind, a, grid, rows, s, nt);
        EDP_MV_TILE_LIST(EDP_CASE)
#define EDP_CASE3(id, kz, nv) EDP_CASE(id, 1, kz, nv)
        EDP_MV3_TILE_LIST(EDP_CASE3)
#undef EDP_CASE3
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

size_t pass_mv_lds_bytes(int tile, int ms, int rows, int ring) {
    switch (tile) {
#define EDP_CASE(id, kx, ky, nv)                                                          \
    case id:                                                                              \
        return ms == MS_WINDOW1 ? mv_lds_bytes_t<MvTileOf<id>::type, 1>(rows, ring)       \
                                : mv_lds_bytes_t<MvTileOf<id>::type, 2>(rows, ring);
        EDP_MV_TILE_LIST(EDP_CASE)
#define EDP_CASE3(id, kz, nv) EDP_CASE(id, 1, kz, nv)
        EDP_MV3_TILE_LIST(EDP_CASE3)
#undef EDP_CASE3
#undef EDP_CASE
    }
    return 0;
}

int pass_mv_capacity(int tile, int kind, int ms, int rows, size_t lds_bytes) {
    int per_cu = 1;
    switch (tile) {
#define EDP_CASE(id, kx, ky, nv)                                                                 \
    case id:                                                                                     \
        per_cu = ms == MS_WINDOW1 ? kind_occ<MvTileOf<id>::type, MS_WINDOW1>(kind, rows, lds_bytes) \
                                  : kind_occ<MvTileOf<id>::type, MS_WINDOW>(kind, rows, lds_bytes);   \
        break;
        EDP_MV_TILE_LIST(EDP_CASE)
#define EDP_CASE3(id, kz, nv) EDP_CASE(id, 1, kz, nv)
        EDP_MV3_TILE_LIST(EDP_CASE3)
#undef EDP_CASE3
#undef EDP_CASE
    }
    int dev = 0, cus = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1;
    return per_cu * cus;
}

// Status words after the scans of a launch class whose last scan formed the labels.
__global__ __launch_bounds__(256) void status_kernel(const InstDesc one, const InstDesc* descs, int32_t ndesc,
                                                     const uint32_t* error) {
    const int32_t v = (error && *error != 0) ? STATUS_TIMEOUT : 0;
    if (ndesc == 0) {
        if (threadIdx.x == 0 && one.status) *one.status = v;
        return;
    }
    for (int32_t i = threadIdx.x; i < ndesc; i += blockDim.x)
        if (descs[i].status) *descs[i].status = v;
}

hipError_t launch_status(const InstDesc& one, const InstDesc* descs, int32_t ndesc, const uint32_t* error,
                         hipStream_t s) {
    hipLaunchKernelGGL(status_kernel, dim3(1), dim3(256), 0, s, one, descs, ndesc, error);
    return hipGetLastError();
}

hipError_t launch_edp_aggregate_mv(int tile, int dtype, const AggArgs& a, int grid, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, kx, ky, nv)                                                                           \
    case id:                                                                                               \
        if (dtype == 1)                                                                                    \
            hipLaunchKernelGGL((edp_aggregate_mv_kernel<MvTileOf<id>::type, int16_t>), dim3(grid), dim3(256), \
                               0, s, a);                                                                   \
        else                                                                                               \
            hipLaunchKernelGGL((edp_aggregate_mv_kernel<MvTileOf<id>::type, int32_t>), dim3(grid), dim3(256), \
                               0, s, a);                                                                   \
        return hipGetLastError();
        EDP_MV_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace edp
