// Scanline DP by min-marginals (Mozerov, arXiv 1410.7922, Sec. 4.1, eqs.
// DP_1D_3 and DP_1D_5) for gfx950.
//
// Every row is a chain.  The forward sweep runs S_1(x) = C(x) + M(S_1(x-1))
// from x = 0 (S_1(0) = C(0)) and stores the forward terms F(x) = M(S_1(x-1))
// (F(0) = 0, the zero boundary); the backward sweep runs S_-1(x) = C(x) +
// M(S_-1(x+1)) from x = W-1 and, at every x, forms the marginal
//   S_Omega(x, v) = F(x, v) + C(x, v) + B(x, v),   B(x) = M(S_-1(x+1)), B(W-1) = 0,
// whose smallest argmin is the label of x (eq. DP_1D_5).  No choice indexes are
// stored and no path is walked back: every label comes out of its own column.
//
// Both sweeps subtract from M(S) the minimum of S, which the minimum search
// returns with no extra reduction: M(S) - min S lies within [0, Vmax], Vmax the
// clip distance of the prior (lambda f(T), twice that for per-dimension
// truncation in two label dimensions), so the forward terms are stored in 16
// bits (the host refuses problems whose Vmax exceeds 65535) and the searched
// vectors stay within the cost range plus Vmax.  Subtracting a constant per
// column shifts S_Omega by a constant per column, which changes neither its
// argmin nor its excess over its minimum; the row optimum is the sum of the
// forward sweep's subtracted minima plus the minimum of its last S.  The minimum search is the scan kernels' (linear RMS or general RMS
// window, one kernel per kind).
#pragma once

#include <type_traits>

#include "edp_device.hpp"
#include "edp_stream.hpp"
#include "edp_internal.hpp"

namespace edp {

__device__ __forceinline__ int32_t off_add(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }

// E forward terms of one lane (contiguous, FT each) at byte offset off; non-temporal loads, like
// those of the costs: the backward sweep reads each once (1.21 -> 1.19 ms on 8192 x 1024 x 64)
template <class FT, int E>
__device__ __forceinline__ void load_terms(__amdgpu_buffer_rsrc_t r, int32_t off, int32_t (&v)[E]) {
    if constexpr (sizeof(FT) == 4) {
        load_vec<E, CPOL_NT>(r, off, v);
    } else if constexpr (E == 1) {
        v[0] = (int32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, CPOL_NT);
    } else {
        int32_t w[E / 2];
        load_vec<E / 2, CPOL_NT>(r, off, w);
#pragma unroll
        for (int k = 0; k < E / 2; ++k) {
            v[2 * k] = w[k] & 0xFFFF;
            v[2 * k + 1] = (int32_t)((uint32_t)w[k] >> 16);
        }
    }
}
template <class FT, int E>
__device__ __forceinline__ void store_terms(__amdgpu_buffer_rsrc_t r, int32_t off, const int32_t (&v)[E]) {
    if constexpr (sizeof(FT) == 4) {
        store_vec<E>(r, off, v);
    } else if constexpr (E == 1) {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v[0], r, off, 0, 0);
    } else {
        int32_t w[E / 2];
#pragma unroll
        for (int k = 0; k < E / 2; ++k)
            w[k] = (int32_t)(((uint32_t)v[2 * k] & 0xFFFFu) | ((uint32_t)v[2 * k + 1] << 16));
        store_vec<E / 2>(r, off, w);
    }
}

// M in place; returns the minimum of h over the vertex (on entry)
template <class T, int MS>
__device__ __forceinline__ int32_t msearch(int32_t (&h)[T::KY][T::KX], const LineIndex<T>& li, const WinPen& wp,
                                           const int32_t clipd, const bool joint, const int32_t lane) {
    if constexpr (MS == MS_LINEAR) return min_search<T>(h, li, clipd, joint, lane);
    else return min_search_window<T, MS == MS_WALK ? 0 : 2>(h, wp, clipd, joint, lane);
}

// FWD: the forward sweep (stores F, writes the row optimum); else the backward sweep (labels and
// the optional marginal excess).  One lane group per row, 64 / G rows per wavefront.
template <class T, class CK, class FT, int PF, int MS, bool FWD>
__global__ __launch_bounds__(256) void dpm_kernel(const DpmArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, E = T::E, QT = T::QT;
    constexpr int RPW = 64 / G;
    constexpr int CB = CostBytes<CK>::value;
    constexpr int CW = CostWords<CK, KX>::value;
    const int32_t lane = lane_id();
    const int32_t grp = lane / G, l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy;
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (wave * RPW >= H) return;                       // whole wavefront past the last row
    const int32_t y = wave * RPW + grp;
    const bool rowok = y < H;
    const bool joint = a.joint != 0;
    const LineIndex<T> li(a.lam, lane);
    const WinPen wp(a.lam, a.trunc, a.qx, a.qy, a.squared != 0);
    const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(a.cost, W * H * Q * CB);
    const __amdgpu_buffer_rsrc_t rs_f = make_rsrc(a.fwd, W * H * QT * (int32_t)sizeof(FT));
    const __amdgpu_buffer_rsrc_t rs_m = make_rsrc(a.marginal, a.marginal ? W * H * Q * 4 : 0);
    const int32_t crow = rowok ? y * W * Q * CB : OOB;
    const int32_t frow = rowok ? (y * W * QT + l * E) * (int32_t)sizeof(FT) : OOB;

    int32_t crun[KY], q[KY][KX];
    bool valid[KY][KX];
#pragma unroll
    for (int ky = 0; ky < KY; ++ky) {
        const int32_t vy = py * KY + ky;
        crun[ky] = (rowok && vy < a.qy && px * KX < a.qx) ? (vy * a.qx + px * KX) * CB : OOB;
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) {
            const int32_t vx = px * KX + kx;
            valid[ky][kx] = rowok && vx < a.qx && vy < a.qy;
            q[ky][kx] = vy * a.qx + vx;
        }
    }
    // step k works on column x(k); the forward sweep takes k = 1 .. W-1, the backward k = 0 .. W-1
    const int32_t k0 = FWD ? 1 : 0;
    auto col = [&](const int32_t k) { return FWD ? k : W - 1 - k; };
    int32_t rc[PF][KY][CW];
    int32_t rf[PF][E];
    auto fetch = [&](const int32_t k, const int u) {
        const bool in = k < W;
        const int32_t x = col(k);
        const int32_t base = in ? off_add(crow, x * Q * CB) : OOB;
#pragma unroll
        for (int ky = 0; ky < KY; ++ky) load_cost_words_nt<CK, KX>(rs_c, in ? off_add(base, crun[ky]) : OOB, rc[u][ky]);
        if constexpr (!FWD) load_terms<FT, E>(rs_f, in ? off_add(frow, x * QT * (int32_t)sizeof(FT)) : OOB, rf[u]);
    };
    // the vector searched next: s on the real labels, PADV on padding labels
    int32_t h[KY][KX];
    auto set_h = [&](const int32_t (&s)[KY][KX]) {
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) h[ky][kx] = valid[ky][kx] ? s[ky][kx] : PADV;
    };

    int64_t offset = 0;
    int32_t bterm[KY][KX];                             // backward: B(x), 0 at x = W-1
    if constexpr (FWD) {
        int32_t c0[KY][CW];
#pragma unroll
        for (int ky = 0; ky < KY; ++ky) load_cost_words_nt<CK, KX>(rs_c, off_add(crow, crun[ky]), c0[ky]);
        const int32_t zero[E] = {};
        store_terms<FT, E>(rs_f, frow, zero);          // F(0) = 0
        int32_t s[KY][KX];
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) s[ky][kx] = cost_elem<CK, KX>(c0[ky], kx);
        set_h(s);
    } else {
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) bterm[ky][kx] = 0;
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) fetch(k0 + u, u);

    auto step = [&](auto tail, const int u, const int32_t k) {
        constexpr bool TAIL = decltype(tail)::value;
        const bool live = !TAIL || k < W;
        const int32_t x = col(k);
        if constexpr (FWD) {
            // F(x) = M(S_1(x-1)) less min S_1(x-1), which the search returns: within [0, Vmax]
            const int32_t g = msearch<T, MS>(h, li, wp, a.clipd, joint, lane);
            int32_t f[E];
#pragma unroll
            for (int e = 0; e < E; ++e) f[e] = (&valid[0][0])[e] ? (&h[0][0])[e] - g : 0;
            store_terms<FT, E>(rs_f, live ? off_add(frow, x * QT * (int32_t)sizeof(FT)) : OOB, f);
            if (live) {
                int32_t s[KY][KX];
#pragma unroll
                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) s[ky][kx] = cost_elem<CK, KX>(rc[u][ky], kx) + f[ky * KX + kx];
                set_h(s);
                offset += g;
            }
        } else {
            // S_Omega(x) = F(x) + C(x) + B(x) and its smallest argmin, found by one minimum over
            // keys ((S_Omega + bias) << ibits) | label (S_Omega + bias >= 0: F, B >= 0, C >= -bias)
            int32_t mg[KY][KX], s[KY][KX];
            int32_t best = 0x7FFFFFFF;
#pragma unroll
            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) {
                    s[ky][kx] = cost_elem<CK, KX>(rc[u][ky], kx) + bterm[ky][kx];
                    mg[ky][kx] = rf[u][ky * KX + kx] + s[ky][kx];
                    const int32_t key = (int32_t)(((uint32_t)(mg[ky][kx] + a.bias) << a.ibits) | (uint32_t)q[ky][kx]);
                    if (valid[ky][kx]) best = imin(best, key);
                }
            best = group_min<T>(best, lane);
            const int32_t qb = best & ((1 << a.ibits) - 1);
            const int32_t mmin = (best >> a.ibits) - a.bias;
            if (live && rowok && l == 0) a.labels[y * W + x] = qb;
#pragma unroll
            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx)
                    store_i32(rs_m, (live && valid[ky][kx]) ? ((y * W + x) * Q + q[ky][kx]) * 4 : OOB,
                              mg[ky][kx] - mmin);
            if (live && x > 0) {
                // B(x-1) = M(S_-1(x)) less min S_-1(x): within [0, Vmax]
                set_h(s);
                const int32_t g = msearch<T, MS>(h, li, wp, a.clipd, joint, lane);
#pragma unroll
                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) bterm[ky][kx] = valid[ky][kx] ? h[ky][kx] - g : 0;
            }
        }
        fetch(k + PF, u);
    };
    const int32_t nsteps = W - k0;
    const int32_t nfull = nsteps / PF;
    int32_t kk = k0;
    for (int32_t r = 0; r < nfull; ++r, kk += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) step(std::false_type{}, u, kk + u);
    }
    if (kk < W) {
#pragma unroll
        for (int u = 0; u < PF; ++u) step(std::true_type{}, u, kk + u);
    }
    if constexpr (FWD) {
        // row optimum: the subtracted minima plus the minimum of the last S_1
        int32_t m = PADV;
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) m = imin(m, h[ky][kx]);
        m = group_min<T>(m, lane);
        if (rowok && l == 0) a.row_energy[y] = offset + m;
    }
}

template <class T>
constexpr int dpm_pf() { return T::E <= 4 ? 8 : 2; }

template <class T, class CK, int MS>
static void run_dpm(const DpmArgs& a, int grid, bool forward, hipStream_t s) {
    if (forward)
        hipLaunchKernelGGL((dpm_kernel<T, CK, uint16_t, dpm_pf<T>(), MS, true>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((dpm_kernel<T, CK, uint16_t, dpm_pf<T>(), MS, false>), dim3(grid), dim3(256), 0, s, a);
}

template <class T, class CK>
static void dpm_ms(const DpmArgs& a, int grid, bool forward, hipStream_t s) {
    if (a.ms == MS_WALK) run_dpm<T, CK, MS_WALK>(a, grid, forward, s);
    else if (a.ms == MS_WINDOW || a.ms == MS_WINDOW1) run_dpm<T, CK, MS_WINDOW>(a, grid, forward, s);
    else run_dpm<T, CK, MS_LINEAR>(a, grid, forward, s);
}

// Per-tile entry point, defined in edp_dpm_a.hip / edp_dpm_b.hip / edp_dpm_c.hip.  Costs are read element
// by element (dtype 1 int16, 2 int32).
template <int ID>
hipError_t dpm_tile(int dtype, const DpmArgs& a, int grid, bool forward, hipStream_t s);

#define EDP_DPM_TILE(id, px, kx, py, ky)                                                           \
    template <>                                                                                     \
    hipError_t dpm_tile<id>(int dtype, const DpmArgs& a, int grid, bool forward, hipStream_t s) {   \
        if (dtype == 1) dpm_ms<Tile<px, kx, py, ky>, int16_t>(a, grid, forward, s);                 \
        else dpm_ms<Tile<px, kx, py, ky>, int32_t>(a, grid, forward, s);                            \
        return hipGetLastError();                                                                   \
    }

}  // namespace edp
