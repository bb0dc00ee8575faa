// Independent-scanline DP with the linear RMS or, for the truncated squared
// prior, the general RMS (Mozerov, arXiv 1410.7922, Sec. 2 eq. One_d / eq. base,
// Sec. 3.1, Sec. 3.2, Sec. 4.1) for gfx950.
//
// Forward sweep.  One lane group (G lanes) per scanline, 64/G scanlines per
// wavefront, the label vector in registers.  Each step computes
//   S(x) = C(x) + M(S(x-1))
// on packed keys key = S * 2^ib + q: every operation of either RMS is a
// min or an addition of a multiple of 2^ib, so running it on keys yields
// M(S)(v) in the high bits and, in the low bits, the smallest label v'
// attaining it -- the optimal choice index of Sec. 4.1, with no second
// search.  The keys stay small because the minimum of S(x-1) is subtracted
// at every step and accumulated separately in int64 (subtracting a constant
// changes no argmin and no tie).
//
// Backtracking.  One workgroup per scanline stages the choice indexes of a
// block of columns in LDS with wide coalesced loads and walks them from
// x = W-1 down to 1.
#include <type_traits>

#include "edp_device.hpp"
#include "edp_stream.hpp"
#include "edp_internal.hpp"

namespace edp {

// key = v * 2^ib + q for 0 <= q < 2^ib (two's complement shift, no signed overflow)
__device__ __forceinline__ int32_t pack(int32_t v, int32_t ib, int32_t q) {
    return (int32_t)(((uint32_t)v << ib) | (uint32_t)q);
}

template <class T, class CK, class PT, int PF, int MS>
__global__ __launch_bounds__(256) void dp_forward_kernel(const DpArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, E = T::E, QT = T::QT;
    constexpr int RPW = 64 / G;
    constexpr int CB = CostBytes<CK>::value;
    const int32_t lane = lane_id();
    const int32_t grp = lane / G, l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy;
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (wave * RPW >= H) return;                       // whole wavefront past the last row
    const int32_t y = wave * RPW + grp;
    const bool rowok = y < H;
    const int32_t ib = a.ibits;
    const int32_t mask = (1 << ib) - 1;
    const int32_t lamk = a.lam << ib, clipk = a.clipd << ib;
    const LineIndex<T> li(lamk, lane);
    const WinPen sp(lamk, a.trunc, a.qx, a.qy, a.squared != 0);   // general RMS window (keys)
    // buffer resources (see the scan kernel): lanes without an operand use offset OOB
    const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(a.cost, W * H * Q * CB);
    const __amdgpu_buffer_rsrc_t rs_p = make_rsrc(a.ptr, W * H * QT * (int32_t)sizeof(PT));
    const int32_t crow = rowok ? y * W * Q * CB : OOB;
    // choice indexes, lane-major: the E labels of a lane are contiguous
    const int32_t prow = rowok ? (y * W * QT + l * E) * (int32_t)sizeof(PT) : OOB;

    int32_t crun[KY], q[KY][KX];                      // cost byte offset of the lane's run of KX labels
    // padding labels hold PADV: key = (key & keep) | pad, a single AND-OR with no branch
    int32_t keep[KY][KX], pad[KY][KX];
#pragma unroll
    for (int ky = 0; ky < KY; ++ky) {
        const int32_t vy = py * KY + ky;
        crun[ky] = (rowok && vy < a.qy && px * KX < a.qx) ? (vy * a.qx + px * KX) * CB : OOB;
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) {
            const int32_t vx = px * KX + kx;
            const bool valid = rowok && vx < a.qx && vy < a.qy;
            q[ky][kx] = vy * a.qx + vx;
            keep[ky][kx] = valid ? -1 : 0;
            pad[ky][kx] = valid ? 0 : PADV;
        }
    }

    constexpr int CW = CostWords<CK, KX>::value;
    int32_t rc[PF][KY][CW];
    // the costs stream through once: non-temporal loads (forward sweep 0.37 -> 0.34 ms on 1 GiB;
    // the choice indexes, which the backtracking reads next, stay cached)
    auto fetch = [&](const int32_t x, int32_t (&c)[KY][CW]) {
        const int32_t base = x < W ? crow + x * Q * CB : OOB;
#pragma unroll
        for (int ky = 0; ky < KY; ++ky) load_cost_words_nt<CK, KX>(rs_c, base + crun[ky], c[ky]);
    };

    int32_t key[KY][KX];
    {
        int32_t c0[KY][CW];
        fetch(0, c0);
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx)
                key[ky][kx] = (pack(cost_elem<CK, KX>(c0[ky], kx), ib, q[ky][kx]) & keep[ky][kx]) | pad[ky][kx];
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) fetch(1 + u, rc[u]);

    int64_t offset = 0;
    const uint32_t mask4 = (uint32_t)mask * 0x01010101u;
    // One step at column x: the choice indexes of x (stored), then S(x) = C(x) + M(S(x-1)).
    // TAIL: the last, partial round of prefetch slots, whose steps past W - 1 change nothing.
    auto step = [&](auto tail, const int u, const int32_t x) {
        constexpr bool TAIL = decltype(tail)::value;
        const bool live = !TAIL || x < W;
        int32_t g;
        if constexpr (MS == MS_LINEAR) g = min_search<T>(key, li, clipk, a.joint != 0, lane);
        else g = min_search_window<T, MS == MS_WALK ? 0 : (MS == MS_WINDOW1 ? 1 : 2)>(key, sp, clipk, a.joint != 0,
                                                                                    lane);
        const int32_t norm = g >> ib;
        if constexpr (sizeof(PT) == 1 && E % 4 == 0) {
            // four choice indexes per dword: low bytes gathered by byte permutes, then masked
#pragma unroll
            for (int e = 0; e < E; e += 4) {
                const int32_t* k = &key[0][0] + e;
                const uint32_t lo = __builtin_amdgcn_perm((uint32_t)k[1], (uint32_t)k[0], 0x0c0c0400u);
                const uint32_t hi = __builtin_amdgcn_perm((uint32_t)k[3], (uint32_t)k[2], 0x0c0c0400u);
                const uint32_t w = __builtin_amdgcn_perm(hi, lo, 0x05040100u) & mask4;
                const int32_t off = live ? prow + (x * QT + e) : OOB;
                __builtin_amdgcn_raw_buffer_store_b32(w, rs_p, off, 0, 0);
            }
        } else {
            uint32_t packed = 0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int32_t k = (&key[0][0])[e];
                packed |= (uint32_t)(k & mask) << (8 * sizeof(PT) * (e % (4 / sizeof(PT))));
                if ((e + 1) % (4 / sizeof(PT)) == 0 || e == E - 1) {
                    const int32_t first = e / (4 / sizeof(PT)) * (4 / sizeof(PT));
                    const int32_t off = live ? prow + (x * QT + first) * (int32_t)sizeof(PT) : OOB;
                    const int32_t nb = (e - first + 1) * (int32_t)sizeof(PT);
                    if (nb == 4) __builtin_amdgcn_raw_buffer_store_b32(packed, rs_p, off, 0, 0);
                    else if (nb == 2) __builtin_amdgcn_raw_buffer_store_b16((uint16_t)packed, rs_p, off, 0, 0);
                    else __builtin_amdgcn_raw_buffer_store_b8((uint8_t)packed, rs_p, off, 0, 0);
                    packed = 0;
                }
            }
        }
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) {
                const int32_t k = key[ky][kx];
                const int32_t v = cost_elem<CK, KX>(rc[u][ky], kx) + (k >> ib) - norm;
                const int32_t nk = (pack(v, ib, q[ky][kx]) & keep[ky][kx]) | pad[ky][kx];
                key[ky][kx] = live ? nk : k;
            }
        offset += live ? norm : 0;
        fetch(x + PF, rc[u]);
    };
    // whole prefetch rounds, then at most one partial round
    const int32_t nfull = (W - 1) / PF;
    int32_t x0 = 1;
    for (int32_t r = 0; r < nfull; ++r, x0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) step(std::false_type{}, u, x0 + u);
    }
    if (x0 < W) {
#pragma unroll
        for (int u = 0; u < PF; ++u) step(std::true_type{}, u, x0 + u);
    }
    int32_t m = PADV;
#pragma unroll
    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) m = imin(m, key[ky][kx]);
    m = group_min<T>(m, lane);
    if (rowok && l == 0) {
        a.row_label[y] = m & mask;
        a.row_energy[y] = offset + (int64_t)(m >> ib);
    }
}

// Backtracking: BT_ROWS scanlines per workgroup, one lane walking each.  The choice
// indexes of a chunk of columns of all the workgroup's scanlines are staged in LDS
// with 16-byte loads by every lane (the block addresses do not depend on the labels);
// then each walking lane follows its scanline through LDS, and the chunk's labels
// leave through LDS in row-contiguous runs.
constexpr int BT_ROWS = 16;

template <class T>
__device__ __forceinline__ int32_t tile_pos(int32_t lab, float inv_qx, int32_t qx) {
    if constexpr (T::PY == 1 && T::KY == 1) {
        return lab;                                  // one label dimension: lane-major order is label order
    } else {
        // lab < 4096 and qx <= 64: the float quotient is within 1e-3 of the true one while
        // (lab + 0.5) / qx stays at least 1 / 128 away from an integer, so the floor is exact
        const int32_t vy = (int32_t)((lab + 0.5f) * inv_qx);
        const int32_t vx = lab - vy * qx;
        const int32_t ppy = vy / T::KY, ky = vy % T::KY, ppx = vx / T::KX, kx = vx % T::KX;
        return (ppy * T::PX + ppx) * T::E + ky * T::KX + kx;
    }
}

template <class T, class PT>
__global__ __launch_bounds__(64) void dp_backtrack_kernel(const BtArgs a) {
    constexpr int QT = T::QT;
    constexpr int V16 = QT * (int)sizeof(PT) / 16;   // 16-byte pieces per column block
    static_assert(QT * sizeof(PT) % 16 == 0, "column blocks of whole 16-byte pieces");
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t C = a.chunk;
    PT* buf = (PT*)smem;                                         // [BT_ROWS][C][QT]
    int32_t* lbuf = (int32_t*)(smem + (size_t)BT_ROWS * C * QT * sizeof(PT));   // [BT_ROWS][C]
    const int32_t t = threadIdx.x;
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy;
    const int32_t y0 = blockIdx.x * BT_ROWS;
    const int32_t nrows = min(BT_ROWS, H - y0);
    const bool walker = t < nrows;
    const float inv_qx = 1.0f / (float)a.qx;
    int32_t lab = walker ? a.row_label[y0 + t] : 0;
    if (walker) a.labels[(size_t)(y0 + t) * W + W - 1] = lab;
    // the choice indexes as one buffer (below 2^31 bytes, checked by the host): pieces
    // outside a scanline's chunk read as zero through an out-of-range offset
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.ptr, (int32_t)((size_t)H * W * QT * sizeof(PT)));
    uint4* dst = (uint4*)buf;
    for (int32_t x1 = W - 1; x1 >= 1; x1 -= C) {
        const int32_t x0 = x1 - C + 1 > 1 ? x1 - C + 1 : 1;
        const int32_t n = x1 - x0 + 1;
        // stage columns x0..x1 of every scanline (row r: n * V16 contiguous pieces), 8 rows x 2
        // pieces per lane in flight at a time
        const int32_t per_row = n * V16;
        for (int32_t ob = 0; ob < per_row; ob += 128) {
            for (int32_t rb = 0; rb < nrows; rb += 8) {
                uint32_t __attribute__((ext_vector_type(4))) v[8][2];
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int32_t r = rb + i, o = ob + t + 64 * j;
                        const int32_t off = (r < nrows && o < per_row)
                                                ? (int32_t)((((size_t)(y0 + r) * W + x0) * V16 + o) * 16)
                                                : OOB;
                        v[i][j] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
                    }
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int32_t r = rb + i, o = ob + t + 64 * j;
                        if (r < nrows && o < per_row) {
                            uint4 w;
                            w.x = v[i][j][0]; w.y = v[i][j][1]; w.z = v[i][j][2]; w.w = v[i][j][3];
                            dst[(size_t)r * C * V16 + o] = w;
                        }
                    }
            }
        }
        __syncthreads();
        if (walker) {
            const PT* rb = buf + (size_t)t * C * QT;
            int32_t* lb = lbuf + t * C;
            for (int32_t x = x1; x >= x0; --x) {
                const int32_t pos = (uint32_t)lab < (uint32_t)Q ? tile_pos<T>(lab, inv_qx, a.qx) : 0;
                lab = rb[(size_t)(x - x0) * QT + pos];
                lb[x - x0] = lab;                    // the label of column x - 1
            }
        }
        __syncthreads();
        for (int32_t k = t; k < nrows * n; k += 64) {
            const int32_t r = k / n, c = k - r * n;
            a.labels[(size_t)(y0 + r) * W + x0 - 1 + c] = lbuf[r * C + c];
        }
        // the next chunk's staging overwrites buf only: lbuf is read above and written after
        // the next barrier
    }
}

template <class T>
constexpr int dp_pf() { return T::E <= 4 ? 8 : 2; }

template <class T, class CK, int MS>
static void run_fwd_ms(const DpArgs& a, int grid, hipStream_t s) {
    if constexpr (T::QT <= 256)
        hipLaunchKernelGGL((dp_forward_kernel<T, CK, uint8_t, dp_pf<T>(), MS>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((dp_forward_kernel<T, CK, uint16_t, dp_pf<T>(), MS>), dim3(grid), dim3(256), 0, s, a);
}

template <class T, class CK>
static hipError_t run_fwd(const DpArgs& a, int grid, hipStream_t s) {
    if (a.ms == MS_WALK) run_fwd_ms<T, CK, MS_WALK>(a, grid, s);
    else if (a.ms == MS_WINDOW1) run_fwd_ms<T, CK, MS_WINDOW1>(a, grid, s);
    else if (a.ms == MS_WINDOW) run_fwd_ms<T, CK, MS_WINDOW>(a, grid, s);
    else run_fwd_ms<T, CK, MS_LINEAR>(a, grid, s);
    return hipGetLastError();
}

// cost kind as for the scan kernel: 1 int16, 2 int32, 3 int16 read in aligned pairs
template <class T>
static hipError_t fwd_kind(int kind, const DpArgs& a, int grid, hipStream_t s) {
    if (kind == 1) return run_fwd<T, int16_t>(a, grid, s);
    if (kind == 3) {
        if constexpr (T::KX % 2 == 0) return run_fwd<T, Pair16>(a, grid, s);
        return hipErrorInvalidValue;
    }
    return run_fwd<T, int32_t>(a, grid, s);
}

template <class T>
static hipError_t run_bt(const BtArgs& a, hipStream_t s) {
    constexpr int pbytes = T::QT <= 256 ? 1 : 2;
    const size_t lds = (size_t)BT_ROWS * a.chunk * (T::QT * pbytes + 4);
    const int grid = (a.H + BT_ROWS - 1) / BT_ROWS;
    if constexpr (T::QT <= 256)
        hipLaunchKernelGGL((dp_backtrack_kernel<T, uint8_t>), dim3(grid), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL((dp_backtrack_kernel<T, uint16_t>), dim3(grid), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_dp_forward(int tile, int kind, const DpArgs& a, int grid, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky) \
    case id:                         \
        return fwd_kind<Tile<px, kx, py, ky>>(kind, a, grid, s);
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dp_backtrack(int tile, const BtArgs& a, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky) \
    case id:                         \
        return run_bt<Tile<px, kx, py, ky>>(a, s);
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace edp
