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

// Wide-vertex tiles of the EDP scans for two-dimensional label spaces: id, KX, KY, NV (ids 16-18,
// then 22-24 after the three-dimensional tiles).
// A vertex takes NV wavefronts; each holds 4 KY label rows of 16 KX labels (lane px of lane
// row r: KX x KY labels), so the tile holds (16 KX) x (4 KY NV) labels and its lane-major
// layout is that of a 16 x (4 NV) lane grid.  Ids follow the single-wavefront tiles.
#define EDP_MV_TILE_LIST(X) \
    X(16, 2, 2, 4)          \
    X(17, 2, 4, 2)          \
    X(18, 1, 2, 2)          \
    X(22, 4, 2, 8)          \
    X(23, 4, 2, 4)          \
    X(24, 2, 2, 8)

// Single-wavefront tiles of three-dimensional label spaces: id, PX, KX, PY, KY, KZ.  Lane
// (px, py) holds the KX x KY labels of the two-dimensional tile at each of the KZ labels
// vz = 0 .. KZ-1 of the third dimension, so a line along z lies inside one lane.  Ids follow
// the wide-vertex tiles.
#define EDP_TILE3_LIST(X)  \
    X(19, 8, 1, 8, 1, 8)   \
    X(20, 4, 1, 4, 1, 4)   \
    X(21, 4, 2, 4, 2, 4)

// Wide-vertex tiles of three-dimensional label spaces: id, KZ, NV.  A vertex of up to
// 8 x 8 x (KZ NV) labels takes NV wavefronts; lane px + 8 py of wavefront w holds the labels
// (px, py, vz) for the KZ labels vz = w KZ ... w KZ + KZ - 1 of the third dimension.
#define EDP_MV3_TILE_LIST(X) \
    X(25, 2, 4)

namespace edp {

constexpr int NUM_TILES = 16;
constexpr int NUM_ALL_TILES = 26;   // every id of the four tile lists is below this
// A wide-vertex tile holds at most this many scanlines per workgroup times its wavefronts
// per vertex: 8 wavefronts (512 lanes).
constexpr int MV_MAX_WAVES = 8;
// compute wavefronts per workgroup of the scan kernel; with its two helper wavefronts a
// workgroup has at most 8, two per SIMD, so each may use half the register file
constexpr int MAX_WAVES = 6;
// The label-window solve: 8 x 8 label frames on tile 13 (8 x 1 by 8 x 1), scan kernel kind 4.
constexpr int WIN_TILE = 13;
constexpr int KIND_WINDOW = 4;
constexpr int WIN_FRAME = 8;
// Minimum searches of the scan and DP kernels (one kernel each, so the step has no branch):
constexpr int MS_LINEAR = 0;     // truncated linear prior: linear RMS (Sec. 3.2)
constexpr int MS_WINDOW = 1;     // general RMS (Sec. 3.1), windows of at most two steps per side, either prior
constexpr int MS_WALK = 2;       // general RMS, any window, truncated squared prior
constexpr int MS_WINDOW1 = 3;    // general RMS, windows of one step per side (T <= 2), either prior

struct TileShape {
    int px, kx, py, ky, kz;
};
TileShape tile_shape(int tile);

// Progress flags and tickets live in the workspace; a scan waits at most this
// many polls (of the order of a second) for its predecessor before giving up
// with an error flag, so a broken schedule ends instead of hanging the device.
constexpr uint32_t SPIN_LIMIT = 1u << 21;
// The second scan of a fused pair waits for whole workgroup bands of the first.
constexpr uint32_t SPIN_LIMIT_BAND = 1u << 22;
// Value of a solve's status word when one of its bounded waits gave up (EDP_E_TIMEOUT of edp.h).
constexpr int32_t STATUS_TIMEOUT = -6;

// One instance of the EDP solve (a batch holds many of them).
struct InstDesc {
    const void* cost;             // [H][W][Q] int16/int32
    int32_t* t[4];                // T arrays +x, -x, +y, -y, [H][W][QT] lane-major
    int32_t* labels;              // [H][W] output labels
    unsigned long long* energy;   // [1] output energy (batched energy kernel), may be null
    uint32_t* flags;              // [3][nsuper]: column progress of the first and the second scan of
                                  // a launch, then the scans completed by each workgroup band
    unsigned long long* hand;     // [2][nsuper-1][W][QT] tagged rows handed between workgroup bands
                                  // (first / second scan of a launch), cleared each solve; or null
    const void* aux;              // label-window solve: int8 frame shifts [H][W][4][2], else null
    const int32_t* centers;       // label-window solve: window centres [H][W][2], else null
    int32_t* status;              // [1] output status word of the solve (0 or STATUS_TIMEOUT), may be null
    int32_t win, qx_full;         // label-window solve: window side, labels along x of the full space
    int32_t W, H, qx, qy;
    int32_t qz;                   // labels along the third label dimension (1: none)
    int32_t lam, clipd, joint, trunc;
    int32_t squared;              // 1: truncated squared prior (clipd = lam trunc^2), 0: truncated linear
    int32_t nbands, nsuper;       // wavefront bands, workgroup bands
    int32_t first_ticket;         // first workgroup band of this instance in its launch
    int32_t first_block;          // first marginal block of this instance
    int32_t first_eblock;         // first energy block of this instance
};

// Status word of every instance of a launch class after its scans (wide tiles, whose last scan
// forms the labels itself): STATUS_TIMEOUT if a wait gave up, else 0.
hipError_t launch_status(const InstDesc& one, const InstDesc* descs, int32_t ndesc, const uint32_t* error,
                         hipStream_t s);

// Locate the instance of a ticket or block: descs sorted by the key, ndesc >= 1;
// by: 0 tickets, 1 marginal blocks, 2 energy blocks.
__device__ __forceinline__ int32_t find_instance(const InstDesc* descs, int32_t ndesc, int32_t key,
                                                 int by_block) {
    int32_t lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        const int32_t first = by_block == 2 ? descs[mid].first_eblock
                              : by_block ? descs[mid].first_block : descs[mid].first_ticket;
        if (first <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A descriptor read from memory with every word made wavefront-uniform, so its
// fields live in scalar registers and control flow on them stays scalar.
__device__ __forceinline__ InstDesc uniform_desc(const InstDesc& src) {
    constexpr int NW32 = (int)(sizeof(InstDesc) / 4);
    int32_t w[NW32];
    __builtin_memcpy(w, &src, sizeof(InstDesc));
#pragma unroll
    for (int i = 0; i < NW32; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    InstDesc d;
    __builtin_memcpy(&d, w, sizeof(InstDesc));
    return d;
}

// Direction set of one EDP scan (P1..P4 of Algorithm 1), T-form: T_k = M(S_k >> 1).
struct PassDir {
    int32_t sx, sy;          // scan direction along x and y (+1 / -1)
    int32_t ka, kb;          // arrays written: ka = x-direction sum, kb = y-direction sum
    int32_t old_a_zero;      // the other x-direction array still holds its initial zeros
    int32_t old_b_zero;      // the other y-direction array still holds its initial zeros
    int32_t b_live;          // the y-direction sum is read by later scans: store it everywhere
    int32_t pass_index;      // scans since the flags were cleared
    int32_t marginal;        // wide tiles, last P4: form the marginal of eq. DP_2D_1 and its smallest
                             // argmin at every vertex (all its terms are at hand) and store no sums
};

// One launch of the scan kernel: one scan, or two consecutive scans that sweep
// the rows in the same order (P1 with P2, P3 with P4), over one instance (ndesc
// 0: the inline `one`) or every instance of a batch class.  Tickets run over
// the workgroup bands of every instance for the first scan, then again for the
// second; a band of the second scan starts once the first scan has finished
// the bands holding its rows and the row after them.
struct PassArgs {
    InstDesc one;
    const InstDesc* descs;
    int32_t ndesc;
    int32_t tickets_per_pass; // workgroup bands of the launch per scan (sum of nsuper)
    int32_t npass;            // 1 or 2
    PassDir dir[2];
    uint32_t* ticket;         // band counter of this launch (zero before the launch)
    uint32_t* error;          // set to 1 when a wait exceeds its limit
    int32_t chunk;            // columns per progress publication (power of two)
    int32_t ring;             // LDS hand-off slots between consecutive wavefronts (power of two)
};

// Marginal and argmin over one instance or a batch class: block b works on
// cells [(b - first_block) * cells_per_block, ...) of its instance.
struct AggArgs {
    InstDesc one;
    const InstDesc* descs;
    int32_t ndesc;
    int32_t cells_per_block;
    const uint32_t* error;   // error word of the scans (nonzero: a wait gave up); the first block of
                             // each instance writes the instance's status word from it
};

struct DpArgs {
    const void* cost;
    void* ptr;               // [H][W][QT] u8 (QT <= 256) or u16 choice indexes
    int32_t* row_label;      // [H] label at x = W-1
    int64_t* row_energy;     // [H]
    int32_t W, H, qx, qy;
    int32_t lam, clipd, joint, trunc;
    int32_t ms;              // minimum search kind MS_*
    int32_t squared;         // truncated squared prior (clipd = lam trunc^2)
    int32_t ibits;           // bits of the label index packed under the value
};

// The min-marginal scanline DP: forward sweep (terms F), then backward sweep (labels).
struct DpmArgs {
    const void* cost;
    void* fwd;               // [H][W][QT] u16 forward terms M(S_1(x-1)) less their minimum, lane-major
    int32_t* labels;         // [H][W]
    int32_t* marginal;       // [H][W][Q] S_Omega less its column minimum, or null
    int64_t* row_energy;     // [H] chain optima
    int32_t W, H, qx, qy;
    int32_t lam, clipd, joint, trunc;
    int32_t ms, squared;     // minimum search kind MS_*, truncated squared prior
    int32_t bias, ibits;     // argmin keys ((S_Omega + bias) << ibits) | label; bias = cost bound
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
    int32_t qz;              // labels along the third label dimension (1: none)
    int32_t lam, trunc, joint, grid4;
    int32_t squared;         // truncated squared prior
    const uint32_t* error;   // the solve's error word (nonzero: energy = INT64_MIN), or null
};

// Energies of every instance of a batch (4-connected): block b works on rows of
// its instance; outputs accumulate into each instance's energy word.
struct BatchEnergyArgs {
    const InstDesc* descs;
    int32_t ndesc;
    int32_t rows_per_block;
    const uint32_t* error;   // the class's error word: nonzero, every energy is INT64_MIN
    int32_t status;          // 1: the first block of each instance also writes its status word
};

// Data cost formation: [H][W][qx*qy] costs of images i0, i1 (and i2 for the composite cost).
struct DsiArgs {
    const uint8_t* i0;
    const uint8_t* i1;
    const uint8_t* i2;       // third view or null
    void* cost;              // int16 or int32 output
    int32_t W, H, qx, qy;
    int32_t ox, oy, sx, sy;  // label (ix, iy) has the displacement (ox + sx ix, oy + sy iy)
    int32_t l2, cmax;
    int32_t vec;             // output 16-byte aligned: vector stores
    double inv_q, inv_w;     // 1 / (qx qy), 1 / W
    // staged-window kernel (set by launch_dsi): segments of seg pixels, nseg per row; the
    // windows are qy rows of pw = seg + qx - 1 pixels from displacement (dxmin, dymin)
    int32_t seg, nseg, pw, dxmin, dxmax, dymin, dymax;
    float inv_qf;            // 1 / (qx qy)
};

// Launchers (return hipSuccess or the launch error).  dtype: 1 int16, 2 int32.
// The scan kernel takes a cost kind instead: 1 int16, 2 int32, 3 int16 read in
// 4-byte aligned pairs (needs an even KX, an even label count, and qx even
// unless qy == 1).
// ms: minimum search kind MS_*
hipError_t launch_edp_pass(int tile, int kind, int split, int ms, const PassArgs& a, int grid, int waves,
                           hipStream_t s);
hipError_t launch_edp_aggregate(int tile, int dtype, const AggArgs& a, int grid, hipStream_t s);
hipError_t launch_edp_aggregate_win(const AggArgs& a, int grid, hipStream_t s);
// label-window solve: compact 8 x 8 frame costs (big outside the window) and frame shifts
hipError_t launch_win_prep(const int32_t* cost, const int32_t* centers, int32_t W, int32_t H, int32_t qx, int32_t qy,
                           int32_t win, int32_t big, int32_t* cw, uint32_t* shifts, hipStream_t s);
hipError_t launch_dp_forward(int tile, int kind, const DpArgs& a, int grid, hipStream_t s);   // a.ms selects the search
hipError_t launch_dp_backtrack(int tile, const BtArgs& a, hipStream_t s);
// dtype: 1 int16, 2 int32 costs
hipError_t launch_dp_marginals(int tile, int dtype, const DpmArgs& a, int grid, bool forward, hipStream_t s);
hipError_t launch_energy(int dtype, const EnergyArgs& a, hipStream_t s);
hipError_t launch_batch_energy(int dtype, const BatchEnergyArgs& a, int grid, hipStream_t s);
hipError_t launch_dsi(const DsiArgs& a, int dtype, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
// the same, plus the n2 (<= 256) words at p2 in the same launch
hipError_t launch_fill_u32_with(uint32_t* p, size_t n, uint32_t* p2, uint32_t n2, uint32_t v, hipStream_t s);
hipError_t launch_sum_rows(const int64_t* rows, int32_t n, int64_t* out, hipStream_t s);
hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, int32_t n, hipStream_t s);

// Resident workgroups of the pass kernel (occupancy x CUs) for a launch shape.
// label-window network kernels (edp_cnn.hip)
hipError_t launch_dsi_motion(const uint8_t* i0, const uint8_t* i1, int32_t W, int32_t H, int32_t r, int32_t cmax,
                             int32_t* out, hipStream_t s);
hipError_t launch_pool(const int32_t* cost, int32_t W, int32_t H, int32_t qx, int32_t qy, int32_t scale,
                       int32_t nbx, int32_t nch, int32_t mode, uint16_t* out, hipStream_t s);
hipError_t launch_conv(int32_t cin, int32_t cout_pad, const uint16_t* in, const uint16_t* w, const float* bias,
                       int32_t h, int32_t wd, int32_t cout_real, int32_t relu, int32_t dil, const uint16_t* mask,
                       int32_t ld, uint16_t* ob, float* of, hipStream_t s);
hipError_t launch_flip(const uint16_t* w, int32_t cin, int32_t cout, int32_t cout_pad, uint16_t* wt, hipStream_t s);
hipError_t launch_wgrad(int32_t cin, int32_t cout_pad, const uint16_t* dy, const uint16_t* x, int32_t h, int32_t wd,
                        int32_t cout_real, int32_t dil, float* dw, hipStream_t s);
hipError_t launch_colsum(const float* a, int32_t rows, int32_t cols, int32_t ld, float* out, hipStream_t s);
hipError_t launch_ce(const float* logits, int32_t n, int32_t ld, const int32_t* tx, const int32_t* ty,
                     int32_t nclass, int32_t win, float* gf, uint16_t* gb, float* loss, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int32_t n, float lr, float b1,
                       float b2, float eps, float clip, int32_t t, hipStream_t s);
hipError_t launch_decode(const float* logits, int32_t h, int32_t w, int32_t ld, int32_t qx, int32_t qy, int32_t win,
                         int32_t nclass, int32_t* centers, hipStream_t s);
hipError_t launch_targets(const int32_t* labels, int32_t W, int32_t H, int32_t qx, int32_t* tx, int32_t* ty,
                          hipStream_t s);
hipError_t launch_recenter(const int32_t* labels, int64_t n, int32_t qx, int32_t qy, int32_t win, int32_t* centers,
                           hipStream_t s);

int pass_capacity(int tile, int kind, int split, int ms, int waves, size_t lds_bytes);
// Wide-vertex scans (tiles NUM_TILES ...): rows = scanlines per workgroup; window kinds only.
// nt: non-temporal loads and stores of the sums (int32 costs)
hipError_t launch_edp_pass_mv(int tile, int kind, int ms, const PassArgs& a, int grid, int rows, hipStream_t s,
                              bool nt);
hipError_t launch_edp_aggregate_mv(int tile, int dtype, const AggArgs& a, int grid, hipStream_t s);
size_t pass_mv_lds_bytes(int tile, int ms, int rows, int ring);
int pass_mv_capacity(int tile, int kind, int ms, int rows, size_t lds_bytes);
// LDS bytes of the pass kernel for a tile, wavefronts per workgroup and ring slots.
size_t pass_lds_bytes(int qt, int waves, int ring);

}  // namespace edp
