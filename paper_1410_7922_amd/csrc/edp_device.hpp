// Device building blocks for gfx950: lane tiles, cross-lane exchange and the
// linear recursive minimum search (Mozerov, arXiv 1410.7922, Sec. 3.2).
//
// A "lane tile" maps the labels of one DSI vertex onto a group of G = PX*PY
// lanes of a 64-wide wavefront.  Lane (px, py) of a group holds the KY x KX
// block of labels vy = py*KY + ky, vx = px*KX + kx, so a line of the label
// space along x lies in consecutive lanes of one lane row and a line along y
// in lanes PX apart.  64 / G groups share a wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace edp {

// Value held by labels outside the label space.  It stays above every real
// value, and adding the largest distance penalty to it cannot overflow int32.
constexpr int32_t PADV = 0x3FFFFFFF;

template <int PX_, int KX_, int PY_, int KY_>
struct Tile {
    static constexpr int PX = PX_, KX = KX_, PY = PY_, KY = KY_;
    static constexpr int G = PX * PY;          // lanes per vertex
    static constexpr int E = KX * KY;          // labels per lane
    static constexpr int QT = G * E;           // padded labels per vertex
    static constexpr int RPW = 64 / G;         // vertices (scanlines) per wavefront
    static_assert(G >= 1 && G <= 64 && (64 % G) == 0, "group must divide the wavefront");
    static_assert((PX & (PX - 1)) == 0 && (PY & (PY - 1)) == 0, "power-of-two lane grid");
};

__device__ __forceinline__ int32_t lane_id() { return (int32_t)__lane_id(); }

// Value of v in lane src (all 64 lanes must execute the call).
__device__ __forceinline__ int32_t from_lane(int32_t v, int32_t src) {
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

// One dimension of the linear RMS on the lane tile: for every line along the
// dimension, the L1 distance transform L(v) = min_v' h(v') + lam |v - v'|
// as the forward pass of eq. L_dec3 and the backward pass of eq. L_dec5
// (lines split over NL lanes, K labels per lane, STEP = lane distance between
// neighbouring lanes of a line), followed by the per-line minimum.
//   val[k]  the K labels of this lane along the line (in/out)
//   pos     this lane's index along the line, 0..NL-1
//   lmin    out: the minimum of the input line (over all NL lanes)
template <int NL, int K, int STEP>
__device__ __forceinline__ void l1_line(int32_t (&val)[K], const int32_t lam, const int32_t pos,
                                        const int32_t lane, int32_t& lmin) {
    int32_t f[K], b[K];
    f[0] = val[0];
#pragma unroll
    for (int k = 1; k < K; ++k) f[k] = imin(val[k], f[k - 1] + lam);
    b[K - 1] = val[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) b[k] = imin(val[k], b[k + 1] + lam);
    int32_t m = val[0];
#pragma unroll
    for (int k = 1; k < K; ++k) m = imin(m, val[k]);
    if constexpr (NL > 1) {
        int32_t tf = f[K - 1];      // value at this lane's last label, scanned forward
        int32_t tb = b[0];          // value at this lane's first label, scanned backward
#pragma unroll
        for (int d = 1; d < NL; d <<= 1) {
            const int32_t uf = from_lane(tf, pos >= d ? lane - d * STEP : lane);
            const int32_t ub = from_lane(tb, pos + d < NL ? lane + d * STEP : lane);
            const int32_t um = from_lane(m, lane ^ (d * STEP));
            tf = imin(tf, uf + lam * (K * d));
            tb = imin(tb, ub + lam * (K * d));
            m = imin(m, um);
        }
        int32_t cf = from_lane(tf, pos >= 1 ? lane - STEP : lane);
        int32_t cb = from_lane(tb, pos + 1 < NL ? lane + STEP : lane);
        if (pos == 0) cf = PADV;
        if (pos == NL - 1) cb = PADV;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            f[k] = imin(f[k], cf + lam * (k + 1));
            b[k] = imin(b[k], cb + lam * (K - k));
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) val[k] = imin(f[k], b[k]);
    lmin = m;
}

// Minimum of v over the G lanes of this lane's group.
template <int G>
__device__ __forceinline__ int32_t group_min(int32_t v, const int32_t lane) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) v = imin(v, from_lane(v, lane ^ d));
    return v;
}

// The minimum search operator M (Sec. 2 eq. M_strf) for the truncated linear
// prior, computed by the linear RMS of Sec. 3.2:
//   joint == false (per-dimension truncation): each label dimension r gets the
//     L1 transform of its lines clipped at (line minimum + clipd), the
//     decomposition of eq. derivation2 applied per dimension;
//   joint == true (truncation of the summed distance, the paper's prior):
//     L_y(L_x(h)) clipped at (min h + clipd), eq. L_dec7.
// h holds the lane's KY x KX labels; padding labels must hold PADV on entry.
// Returns min h over the whole vertex (the group).
template <class T>
__device__ __forceinline__ int32_t min_search(int32_t (&h)[T::KY][T::KX], const int32_t lam,
                                              const int32_t clipd, const bool joint,
                                              const int32_t lane) {
    const int32_t l = lane % T::G;
    const int32_t px = l % T::PX, py = l / T::PX;
    int32_t rowmin = PADV;
#pragma unroll
    for (int ky = 0; ky < T::KY; ++ky) {
        int32_t lm;
        l1_line<T::PX, T::KX, 1>(h[ky], lam, px, lane, lm);
        rowmin = imin(rowmin, lm);
        if (!joint) {
#pragma unroll
            for (int kx = 0; kx < T::KX; ++kx) h[ky][kx] = imin(h[ky][kx], lm + clipd);
        }
    }
    // rowmin: min over this lane's lines of the input; the global min needs the y lanes too.
    int32_t gmin = rowmin;
#pragma unroll
    for (int d = 1; d < T::PY; d <<= 1) gmin = imin(gmin, from_lane(gmin, lane ^ (d * T::PX)));
    if constexpr (T::PY * T::KY > 1) {
#pragma unroll
        for (int kx = 0; kx < T::KX; ++kx) {
            int32_t col[T::KY];
#pragma unroll
            for (int ky = 0; ky < T::KY; ++ky) col[ky] = h[ky][kx];
            int32_t lm;
            l1_line<T::PY, T::KY, T::PX>(col, lam, py, lane, lm);
#pragma unroll
            for (int ky = 0; ky < T::KY; ++ky) h[ky][kx] = joint ? col[ky] : imin(col[ky], lm + clipd);
        }
    }
    if (joint) {
#pragma unroll
        for (int ky = 0; ky < T::KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < T::KX; ++kx) h[ky][kx] = imin(h[ky][kx], gmin + clipd);
    }
    return gmin;
}

}  // namespace edp
