// EDP scans and marginal (Mozerov, arXiv 1410.7922, Sec. 4.2) for gfx950.
//
// T-form.  Every use of a sum S_k in eq. DP_2D_base and eq. DP_2D_1 is
// M(S_k(x_k) / 2), so the kernels store T_k(x) = M(S_k(x) >> 1) instead of
// S_k.  A scan with directions (sx, sy) computes, at vertex (x, y),
//   A   = C + T_a(x - sx, y) + T_b(x, y - sy)          (this scan's own sums)
//   S_a = A + T_-b(x, y + sy) - T_-a(x + sx, y)        (k' = a: sum over K \ {-a})
//   S_b = A + T_-a(x + sx, y) - T_-b(x, y + sy)        (k' = b: sum over K \ {-b})
//   T_a = M(S_a >> 1),  T_b = M(S_b >> 1)
// with a = sx * x-axis, b = sy * y-axis, T = 0 off the grid and before the
// first scan (all S_k start at 0 and M(0) = 0).  The data cost C is added as
// in the one-dimensional forms (eq. base, eq. DP_1D_3).
//
// Schedule.  Inside a scan vertex (x, y) depends on (x - sx, y) and
// (x, y - sy): a 2D wavefront.  A wavefront of 64 lanes owns a band of
// 64/G consecutive scanlines (G lanes per vertex); its lane groups run one
// column apart, so the T_b a group produces at step s is handed to the group
// below at step s + 1 with one cross-lane read.  Bands are taken in scan
// order from a ticket counter, so the band a wavefront waits on is always
// held by a wavefront that is already running; the last scanline of a band
// publishes its progress every `chunk` columns (release at agent scope) and
// the next band's first scanline reads it from memory after an acquire.
// Operands that do not depend on the scan (C and the two "old" arrays) are
// prefetched PF steps ahead in a register ring.
#include "edp_device.hpp"
#include "edp_internal.hpp"

namespace edp {

template <class T, class CT, int PF>
__global__ __launch_bounds__(64) void edp_pass_kernel(const PassArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, RPW = T::RPW, QT = T::QT;
    const int32_t lane = lane_id();
    const int32_t grp = lane / G, l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy;
    const CT* __restrict__ cost = (const CT*)a.cost;
    int32_t* __restrict__ Ta = a.t[a.ka];
    int32_t* __restrict__ Tb = a.t[a.kb];
    const int32_t* __restrict__ Tma = a.t[a.ka ^ 1];
    const int32_t* __restrict__ Tmb = a.t[a.kb ^ 1];

    int32_t coff[KY][KX];
    bool valid[KY][KX];
#pragma unroll
    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) {
            const int32_t vy = py * KY + ky, vx = px * KX + kx;
            valid[ky][kx] = vx < a.qx && vy < a.qy;
            coff[ky][kx] = vy * a.qx + vx;
        }

    for (;;) {
        int32_t band = 0;
        if (lane == 0) band = (int32_t)atomicAdd(a.ticket, 1u);
        band = __builtin_amdgcn_readfirstlane(band);
        if (band >= a.nbands) break;

        const int32_t j = band * RPW + grp;            // scan-order row index
        const bool rowok = j < H;
        const int32_t y = a.sy > 0 ? j : H - 1 - j;
        const int32_t yp = y - a.sy;                   // previous row in scan order
        const int32_t yn = y + a.sy;                   // next row in scan order
        const bool has_next = j + 1 < H;
        const bool global_b = band > 0;                // group 0 reads the band above from memory
        uint32_t seen = 0;                             // columns the band above has published
        const int32_t nsteps = W + RPW - 1;

        int32_t rc[PF][KY][KX], rma[PF][KY][KX], rmb[PF][KY][KX], rb[PF][KY][KX];
        int32_t carry[KY][KX], tbout[KY][KX];
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) carry[ky][kx] = tbout[ky][kx] = 0;

        // Issue the loads of step t into ring slot u.
        auto fetch = [&](const int32_t t, int32_t (&c)[KY][KX], int32_t (&ma)[KY][KX],
                         int32_t (&mb)[KY][KX], int32_t (&gb)[KY][KX]) {
            if (global_b && t < W) {                   // wave-uniform wait for the band above
                const uint32_t need = (uint32_t)t + 1;
                if (seen < need) {
                    uint32_t got = 0;
                    if (lane == 0) {
                        uint32_t v = 0, spins = 0;
                        for (;;) {
                            v = __hip_atomic_load(a.flags + band - 1, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                            if (v >= a.epoch + need) break;
                            // give up (and let every other waiter give up) instead of hanging
                            if (++spins > SPIN_LIMIT ||
                                __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                __hip_atomic_store(a.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                v = a.epoch + (uint32_t)W;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        got = v - a.epoch;
                    }
                    seen = __builtin_amdgcn_readfirstlane(got);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            const int32_t i = t - grp;
            const bool act = rowok && i >= 0 && i < W;
            const int32_t x = a.sx > 0 ? i : W - 1 - i;
            const int32_t xa = x + a.sx;
            const bool ina = act && xa >= 0 && xa < W && !a.old_a_zero;
            const bool inb = act && has_next && !a.old_b_zero;
            const bool ing = act && global_b && grp == 0;
            const size_t cell = (size_t)y * W + x;
            const CT* cc = cost + cell * Q;
            const int32_t* pa = Tma + ((size_t)y * W + xa) * QT + l;
            const int32_t* pb = Tmb + ((size_t)yn * W + x) * QT + l;
            const int32_t* pg = Tb + ((size_t)yp * W + x) * QT + l;
#pragma unroll
            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) {
                    const int e = (ky * KX + kx) * G;
                    c[ky][kx] = (act && valid[ky][kx]) ? (int32_t)cc[coff[ky][kx]] : 0;
                    ma[ky][kx] = ina ? pa[e] : 0;
                    mb[ky][kx] = inb ? pb[e] : 0;
                    gb[ky][kx] = ing ? pg[e] : 0;
                }
        };

#pragma unroll
        for (int u = 0; u < PF; ++u) fetch(u, rc[u], rma[u], rmb[u], rb[u]);

        for (int32_t s0 = 0; s0 < nsteps; s0 += PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int32_t s = s0 + u;
                if (s < nsteps) {
                    const int32_t i = s - grp;
                    const bool act = rowok && i >= 0 && i < W;
                    const int32_t x = a.sx > 0 ? i : W - 1 - i;
                    int32_t ha[KY][KX], hb[KY][KX];
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx) {
                            int32_t mbv = from_lane(tbout[ky][kx], (lane - G) & 63);
                            if (grp == 0) mbv = rb[u][ky][kx];
                            const int32_t A = rc[u][ky][kx] + carry[ky][kx] + mbv;
                            const int32_t d = rmb[u][ky][kx] - rma[u][ky][kx];
                            ha[ky][kx] = valid[ky][kx] ? ((A + d) >> 1) : PADV;
                            hb[ky][kx] = valid[ky][kx] ? ((A - d) >> 1) : PADV;
                        }
                    min_search<T>(ha, a.lam, a.clipd, a.joint != 0, lane);
                    min_search<T>(hb, a.lam, a.clipd, a.joint != 0, lane);
                    if (act) {
                        int32_t* oa = Ta + ((size_t)y * W + x) * QT + l;
                        int32_t* ob = Tb + ((size_t)y * W + x) * QT + l;
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                            for (int kx = 0; kx < KX; ++kx) {
                                const int e = (ky * KX + kx) * G;
                                oa[e] = ha[ky][kx];
                                ob[e] = hb[ky][kx];
                                carry[ky][kx] = ha[ky][kx];
                            }
                    }
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx) tbout[ky][kx] = hb[ky][kx];
                    // publish the band's progress to the band below
                    if (band + 1 < a.nbands) {
                        const int32_t il = s - (RPW - 1);
                        if (il >= 0 && il < W && (((il + 1) % a.chunk) == 0 || il == W - 1)) {
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                            if (lane == 0)
                                __hip_atomic_store(a.flags + band, a.epoch + (uint32_t)(il + 1),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                    if (s + PF < nsteps) fetch(s + PF, rc[u], rma[u], rmb[u], rb[u]);
                }
            }
        }
    }
}

template <class T, class CT>
__global__ __launch_bounds__(256) void edp_aggregate_kernel(const AggArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, RPW = T::RPW, QT = T::QT;
    const int32_t lane = lane_id();
    const int32_t grp = lane / G, l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy;
    const CT* __restrict__ cost = (const CT*)a.cost;
    const int32_t wave = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int32_t nwaves = (int32_t)((gridDim.x * blockDim.x) >> 6);
    const int32_t cells = W * H;
    for (int32_t base = wave * RPW; base < cells; base += nwaves * RPW) {
        const int32_t cell = base + grp;
        const bool ok = cell < cells;
        const int32_t y = ok ? cell / W : 0, x = ok ? cell % W : 0;
        int32_t best = 0x7FFFFFFF, bq = 0x7FFFFFFF;
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) {
                const int32_t vy = py * KY + ky, vx = px * KX + kx;
                if (ok && vx < a.qx && vy < a.qy) {
                    const int32_t q = vy * a.qx + vx;
                    const int e = (ky * KX + kx) * G + l;
                    int32_t v = (int32_t)cost[(size_t)cell * Q + q];
                    if (x > 0) v += a.t[0][(size_t)(cell - 1) * QT + e];
                    if (x + 1 < W) v += a.t[1][(size_t)(cell + 1) * QT + e];
                    if (y > 0) v += a.t[2][(size_t)(cell - W) * QT + e];
                    if (y + 1 < H) v += a.t[3][(size_t)(cell + W) * QT + e];
                    if (v < best || (v == best && q < bq)) { best = v; bq = q; }
                }
            }
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const int32_t ob = from_lane(best, lane ^ d);
            const int32_t oq = from_lane(bq, lane ^ d);
            if (ob < best || (ob == best && oq < bq)) { best = ob; bq = oq; }
        }
        if (ok && l == 0) a.labels[cell] = bq;
    }
}

// Prefetch depth by labels per lane: more labels per lane, fewer ring slots.
template <class T>
constexpr int pass_pf() { return T::E <= 2 ? 4 : (T::E <= 4 ? 2 : 1); }

template <class T, class CT>
static hipError_t run_pass(const PassArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((edp_pass_kernel<T, CT, pass_pf<T>()>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <class T, class CT>
static hipError_t run_agg(const AggArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((edp_aggregate_kernel<T, CT>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class T, class CT>
static int pass_occupancy() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, edp_pass_kernel<T, CT, pass_pf<T>()>, 64, 0) !=
        hipSuccess)
        blocks = 1;
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_edp_pass(int tile, int dtype, const PassArgs& a, int grid, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                                   \
    case id:                                                                           \
        return dtype == 1 ? run_pass<Tile<px, kx, py, ky>, int16_t>(a, grid, s)        \
                          : run_pass<Tile<px, kx, py, ky>, int32_t>(a, grid, s);
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_edp_aggregate(int tile, int dtype, const AggArgs& a, int grid, hipStream_t s) {
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                                   \
    case id:                                                                           \
        return dtype == 1 ? run_agg<Tile<px, kx, py, ky>, int16_t>(a, grid, s)         \
                          : run_agg<Tile<px, kx, py, ky>, int32_t>(a, grid, s);
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

int pass_capacity(int tile, int dtype) {
    static int cache[NUM_TILES][2] = {};
    const int di = dtype == 1 ? 0 : 1;
    if (tile < 0 || tile >= NUM_TILES) return 1;
    if (cache[tile][di] == 0) {
        int per_cu = 1;
        switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                                              \
    case id:                                                                                      \
        per_cu = dtype == 1 ? pass_occupancy<Tile<px, kx, py, ky>, int16_t>()                     \
                            : pass_occupancy<Tile<px, kx, py, ky>, int32_t>();                    \
        break;
            EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
        }
        int dev = 0, cus = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 1;
        cache[tile][di] = per_cu * cus;
    }
    return cache[tile][di];
}

}  // namespace edp
