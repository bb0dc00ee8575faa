// Internal interface between the C ABI (edp_api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// Lane tiles compiled into the library: id, PX, KX, PY, KY.  A tile holds
// (PX*KX) x (PY*KY) labels on PX*PY lanes.
#define EDP_TILE_LIST(X) \
    X(0, 16, 1, 1, 1)    \
    X(1, 32, 1, 1, 1)    \
    X(2, 64, 1, 1, 1)    \
    X(3, 16, 2, 1, 1)    \
    X(4, 8, 4, 1, 1)     \
    X(5, 16, 4, 1, 1)    \
    X(6, 32, 2, 1, 1)    \
    X(7, 64, 4, 1, 1)    \
    X(8, 32, 8, 1, 1)    \
    X(9, 4, 4, 4, 4)     \
    X(10, 4, 4, 16, 1)   \
    X(11, 8, 2, 8, 2)    \
    X(12, 8, 4, 8, 4)    \
    X(13, 8, 1, 8, 1)    \
    X(14, 4, 2, 4, 2)    \
    X(15, 4, 8, 16, 2)

namespace edp {

constexpr int NUM_TILES = 16;

struct TileShape {
    int px, kx, py, ky;
};
TileShape tile_shape(int tile);

// Progress flags and tickets live in the workspace; a scan waits at most this
// many polls (of the order of a second) for its predecessor before giving up
// with an error flag, so a broken schedule ends instead of hanging the device.
constexpr uint32_t SPIN_LIMIT = 1u << 21;

// One EDP scan (P1..P4) over the grid, T-form: T_k = M(S_k >> 1).
struct PassArgs {
    const void* cost;        // [H][W][Q] int16/int32
    int32_t* t[4];           // T arrays +x, -x, +y, -y in tile layout [H][W][QT]
    uint32_t* flags;         // [nsuper] progress, monotone across the scans of one solve
    uint32_t* ticket;        // band counter of this scan (zero before the scan)
    uint32_t* error;         // set to 1 when a wait exceeds SPIN_LIMIT
    int32_t W, H, qx, qy;
    int32_t lam, clipd, joint;
    int32_t sx, sy;          // scan direction along x and y (+1 / -1)
    int32_t ka, kb;          // arrays written: ka = x-direction sum, kb = y-direction sum
    int32_t old_a_zero;      // the other x-direction array still holds its initial zeros
    int32_t old_b_zero;      // the other y-direction array still holds its initial zeros
    uint32_t epoch;          // flag base of this scan
    int32_t chunk;           // columns per progress publication
    int32_t nbands;          // scanline bands (one wavefront each)
    int32_t nsuper;          // workgroup bands (waves per workgroup consecutive bands each)
    int32_t b_live;          // the y-direction sum is read by later scans: store it everywhere
    int32_t ring;            // LDS hand-off slots between consecutive wavefronts of a workgroup
};

struct AggArgs {
    const void* cost;
    const int32_t* t[4];
    int32_t* labels;
    int32_t W, H, qx, qy;
};

struct DpArgs {
    const void* cost;
    void* ptr;               // [H][W][QT] u8 (QT <= 256) or u16 choice indexes
    int32_t* row_label;      // [H] label at x = W-1
    int64_t* row_energy;     // [H]
    int32_t W, H, qx, qy;
    int32_t lam, clipd, joint;
    int32_t ibits;           // bits of the label index packed under the value
};

struct BtArgs {
    const void* ptr;
    const int32_t* row_label;
    int32_t* labels;
    int32_t W, H, qx, qy;
    int32_t chunk;           // columns staged in LDS at a time
};

struct EnergyArgs {
    const void* cost;
    const int32_t* labels;
    unsigned long long* energy;
    unsigned long long* invalid;
    int32_t W, H, qx, qy;
    int32_t lam, trunc, joint, grid4;
};

// Launchers (return hipSuccess or the launch error).  dtype: 1 int16, 2 int32.
// The scan kernel takes a cost kind instead: 1 int16, 2 int32, 3 int16 read in
// 4-byte aligned pairs (needs an even KX, an even label count, and qx even
// unless qy == 1).
hipError_t launch_edp_pass(int tile, int kind, int split, const PassArgs& a, int grid, int waves,
                           hipStream_t s);
hipError_t launch_edp_aggregate(int tile, int dtype, const AggArgs& a, int grid, hipStream_t s);
hipError_t launch_dp_forward(int tile, int dtype, const DpArgs& a, int grid, hipStream_t s);
hipError_t launch_dp_backtrack(int tile, const BtArgs& a, hipStream_t s);
hipError_t launch_energy(int dtype, const EnergyArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_sum_rows(const int64_t* rows, int32_t n, int64_t* out, hipStream_t s);
hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, int32_t n, hipStream_t s);

// Resident workgroups of the pass kernel (occupancy x CUs) for a launch shape.
int pass_capacity(int tile, int kind, int split, int waves, size_t lds_bytes);
// LDS bytes of the pass kernel for a tile, wavefronts per workgroup and ring slots.
size_t pass_lds_bytes(int qt, int waves, int ring);

}  // namespace edp
