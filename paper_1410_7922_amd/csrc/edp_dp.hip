// Independent-scanline DP with the linear RMS (Mozerov, arXiv 1410.7922,
// Sec. 2 eq. One_d / eq. base, Sec. 3.2, Sec. 4.1) for gfx950.
//
// Forward sweep.  One lane group (G lanes) per scanline, 64/G scanlines per
// wavefront, the label vector in registers.  Each step computes
//   S(x) = C(x) + M(S(x-1))
// on packed keys key = S * 2^ib + q: every operation of the linear RMS is a
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
#include "edp_device.hpp"
#include "edp_internal.hpp"

namespace edp {

// key = v * 2^ib + q for 0 <= q < 2^ib (two's complement shift, no signed overflow)
__device__ __forceinline__ int32_t pack(int32_t v, int32_t ib, int32_t q) {
    return (int32_t)(((uint32_t)v << ib) | (uint32_t)q);
}

template <class T, class CT, class PT, int PF>
__global__ __launch_bounds__(256) void dp_forward_kernel(const DpArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, E = T::E, QT = T::QT;
    constexpr int RPW = 64 / G;
    constexpr int CB = (int)sizeof(CT);
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
    // buffer resources (see the scan kernel): lanes without an operand use offset OOB
    const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(a.cost, W * H * Q * CB);
    const __amdgpu_buffer_rsrc_t rs_p = make_rsrc(a.ptr, W * H * QT * (int32_t)sizeof(PT));
    const int32_t crow = rowok ? y * W * Q * CB : OOB;
    // choice indexes, lane-major: the E labels of a lane are contiguous
    const int32_t prow = rowok ? (y * W * QT + l * E) * (int32_t)sizeof(PT) : OOB;

    int32_t coffb[KY][KX], q[KY][KX];
    bool valid[KY][KX];
#pragma unroll
    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) {
            const int32_t vy = py * KY + ky, vx = px * KX + kx;
            valid[ky][kx] = rowok && vx < a.qx && vy < a.qy;
            q[ky][kx] = vy * a.qx + vx;
            coffb[ky][kx] = valid[ky][kx] ? q[ky][kx] * CB : OOB;
        }

    int32_t rc[PF][KY][KX];
    auto fetch = [&](const int32_t x, int32_t (&c)[KY][KX]) {
        const int32_t base = x < W ? crow + x * Q * CB : OOB;
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) c[ky][kx] = load_cost<CT>(rs_c, base + coffb[ky][kx]);
    };

    int32_t key[KY][KX];
    {
        int32_t c0[KY][KX];
        fetch(0, c0);
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx)
                key[ky][kx] = valid[ky][kx] ? pack(c0[ky][kx], ib, q[ky][kx]) : PADV;
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) fetch(1 + u, rc[u]);

    int64_t offset = 0;
    // whole prefetch rounds (steps past W - 1 change nothing), see the scan kernel
    const int32_t xend = 1 + (W - 1 + PF - 1) / PF * PF;
    for (int32_t x0 = 1; x0 < xend; x0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int32_t x = x0 + u;
            const bool live = x < W;
            const int32_t g = min_search<T>(key, li, clipk, a.joint != 0, lane);
            const int32_t norm = g >> ib;
            uint32_t packed = 0;
#pragma unroll
            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) {
                    const int32_t k = key[ky][kx];
                    packed |= (uint32_t)(k & mask) << (8 * sizeof(PT) * ((ky * KX + kx) % (4 / sizeof(PT))));
                    if (((ky * KX + kx) + 1) % (4 / sizeof(PT)) == 0 || (ky * KX + kx) == E - 1) {
                        const int32_t first = (ky * KX + kx) / (4 / sizeof(PT)) * (4 / sizeof(PT));
                        const int32_t off = live ? prow + (x * QT + first) * (int32_t)sizeof(PT) : OOB;
                        const int32_t nb = ((ky * KX + kx) - first + 1) * (int32_t)sizeof(PT);
                        if (nb == 4) __builtin_amdgcn_raw_buffer_store_b32(packed, rs_p, off, 0, 0);
                        else if (nb == 2) __builtin_amdgcn_raw_buffer_store_b16((uint16_t)packed, rs_p, off, 0, 0);
                        else __builtin_amdgcn_raw_buffer_store_b8((uint8_t)packed, rs_p, off, 0, 0);
                        packed = 0;
                    }
                    const int32_t v = rc[u][ky][kx] + (k >> ib) - norm;
                    const int32_t nk = valid[ky][kx] ? pack(v, ib, q[ky][kx]) : PADV;
                    key[ky][kx] = live ? nk : key[ky][kx];
                }
            offset += live ? norm : 0;
            fetch(x + PF, rc[u]);
        }
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

template <class T, class PT>
__global__ __launch_bounds__(64) void dp_backtrack_kernel(const BtArgs a) {
    constexpr int QT = T::QT;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint16_t tab[4096];
    PT* buf = (PT*)smem;
    const int32_t y = blockIdx.x;
    const int32_t t = threadIdx.x;
    const int32_t W = a.W, Q = a.qx * a.qy;
    for (int32_t q = t; q < Q; q += 64) {
        const int32_t vy = q / a.qx, vx = q % a.qx;
        const int32_t ppy = vy / T::KY, ky = vy % T::KY, ppx = vx / T::KX, kx = vx % T::KX;
        tab[q] = (uint16_t)((ppy * T::PX + ppx) * T::E + ky * T::KX + kx);
    }
    int32_t lab = a.row_label[y];
    int32_t* out = a.labels + (size_t)y * W;
    if (t == 0) out[W - 1] = lab;
    __syncthreads();
    const size_t rowbase = (size_t)y * W * QT;
    for (int32_t x1 = W - 1; x1 >= 1; x1 -= a.chunk) {
        const int32_t x0 = x1 - a.chunk + 1 > 1 ? x1 - a.chunk + 1 : 1;
        const size_t nbytes = (size_t)(x1 - x0 + 1) * QT * sizeof(PT);
        const uint4* src = (const uint4*)((const PT*)a.ptr + rowbase + (size_t)x0 * QT);
        uint4* dst = (uint4*)buf;
        for (size_t k = t; k < nbytes / 16; k += 64) dst[k] = src[k];
        __syncthreads();
        if (t == 0) {
            for (int32_t x = x1; x >= x0; --x) {
                const int32_t pos = (uint32_t)lab < (uint32_t)Q ? tab[lab] : 0;
                lab = buf[(size_t)(x - x0) * QT + pos];
                out[x - 1] = lab;
            }
        }
        __syncthreads();
    }
}

template <class T>
constexpr int dp_pf() { return T::E <= 4 ? 4 : 2; }

template <class T, class CT>
static hipError_t run_fwd(const DpArgs& a, int grid, hipStream_t s) {
    if (T::QT <= 256)
        hipLaunchKernelGGL((dp_forward_kernel<T, CT, uint8_t, dp_pf<T>()>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((dp_forward_kernel<T, CT, uint16_t, dp_pf<T>()>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class T>
static hipError_t run_bt(const BtArgs& a, hipStream_t s) {
    const size_t lds = (size_t)a.chunk * T::QT * (T::QT <= 256 ? 1 : 2);
    if (T::QT <= 256)
        hipLaunchKernelGGL((dp_backtrack_kernel<T, uint8_t>), dim3(a.H), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL((dp_backtrack_kernel<T, uint16_t>), dim3(a.H), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_dp_forward(int tile, int dtype, const DpArgs& a, int grid, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                                  \
    case id:                                                                          \
        return dtype == 1 ? run_fwd<Tile<px, kx, py, ky>, int16_t>(a, grid, s)        \
                          : run_fwd<Tile<px, kx, py, ky>, int32_t>(a, grid, s);
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
