// EDP scans (Mozerov, arXiv 1410.7922, Sec. 4.2) with a vertex spread over several
// wavefronts, for two- and three-dimensional label spaces.
//
// The scans compute the same T-form recursion as edp_pass_kernel (see there):
//   A   = C + T_a(x - sx, y) + T_b(x, y - sy)
//   T_a = M((A + T_-b(x, y + sy) - T_-a(x + sx, y)) >> 1)
//   T_b = M((A + T_-a(x + sx, y) - T_-b(x, y + sy)) >> 1)
// The step of a scan is a chain: T_a of one vertex feeds the next vertex of the
// scanline, so the time of a scan is its number of dependent steps times the
// latency of one step.  With all labels of a vertex on one wavefront that
// latency is the whole minimum search of a large label space.  Here the labels
// of a vertex lie on NV wavefronts, each holding a slab of label rows:
//
//  * wavefront w holds the label rows vy = w * SY ... (w + 1) * SY - 1, SY = 4 KY;
//    in it, lane row r (16 lanes) holds rows w SY + r KY ... + KY - 1 and lane px of
//    the row the labels vx = px KX ... px KX + KX - 1 (so the lane-major order of a
//    vertex is that of a 16 x (4 NV) lane grid with KX x KY labels per lane);
//  * the minimum search runs separably (eq. M_decmp): the window along x (eq.
//    M_decmp1) stays inside a 16-lane row (DPP moves); for the window along y the
//    wavefronts of the vertex write the x results of the label rows next to their
//    slab edges, and their column minima, to an exchange plane in LDS, meet at a
//    counter, and read the rows they need;
//  * everything else of the step (the sums, the loads and stores, the hand-off of
//    T_b to the next scanline) concerns the wavefront's own slab only.
//
// Three label dimensions (MvTile3): wavefront w holds slices of the third dimension,
// all 8 x 8 (x, y) labels of each on its lanes; the windows along x and y run inside
// the wavefront, the one along z through the exchange plane, which then holds whole
// slices.
//
// A workgroup holds RW consecutive scanlines of one scan, each on NV wavefronts.
// Scanline k hands T_b to scanline k + 1 through an LDS ring per wavefront slab;
// the last scanline of the workgroup stores it as tagged 64-bit words (value and
// a tag naming scan, workgroup band and column; word-major, so every store is a
// whole run of sectors) that two helper wavefronts of the next workgroup poll, two
// row buffers per scan of a launch used alternately by consecutive workgroup bands (a band writes column c only after the band below
// the previous user of the buffer has read column c: it needs that band's result
// at column c first).  Workgroups take bands in scan order from a ticket counter,
// as in edp_pass_kernel; the fused second scan of a launch waits for whole bands
// of the first.  Only the general RMS window kinds (at most two steps per side)
// are compiled here.
#pragma once
#include "edp_pass_kernel.hpp"

namespace edp {

template <int KX_, int KY_, int NV_>
struct MvTile {
    static constexpr bool D3 = false;
    static constexpr int KX = KX_, KY = KY_, NV = NV_;
    static constexpr int QXP = 16 * KX;           // labels along x: one 16-lane row
    static constexpr int SY = 4 * KY;             // label rows per wavefront
    static constexpr int QYP = NV * SY;           // labels along y
    static constexpr int E = KX * KY;             // labels per lane
    static constexpr int QT = QXP * QYP;          // labels per vertex (padded)
    using Lane = Tile<16, KX, 4, KY>;             // layout inside one wavefront
    // exchange plane: PH rows (y) of PW words (x), then the column minima of each wavefront
    static constexpr int PW = QXP, PH = QYP, CM = NV * QXP;
};

// A vertex of a three-dimensional label space on NV wavefronts: wavefront w holds the slices
// vz = w KZ ... w KZ + KZ - 1 of the 8 x 8 (x, y) labels, lane px + 8 py the labels (px, py)
// of its KZ slices (a tile of three-dimensional label spaces, Tile<8, 1, 8, 1, KZ>, per
// wavefront).  The windows along x and y stay inside the wavefront; the window along z runs
// across the wavefronts through an exchange plane of whole slices.  The label arrays of the
// kernel take the slices as rows (KY = KZ, KX = 1).
template <int KZ_, int NV_>
struct MvTile3 {
    static constexpr bool D3 = true;
    static constexpr int KX = 1, KY = KZ_, NV = NV_;
    static constexpr int QXP = 8, QYP = 8, QZP = NV * KZ_;
    static constexpr int SY = 0;                  // (two-dimensional layouts only)
    static constexpr int E = KZ_;
    static constexpr int QT = QXP * QYP * QZP;
    using Lane = Tile<8, 1, 8, 1, KZ_>;
    // exchange plane: PH slices of 64 words, then each wavefront's per-lane minimum over its
    // slices [NV][64] and its minimum over all its labels [NV]
    static constexpr int PW = 64, PH = QZP, CM = NV * 64 + NV;
};

// LDS words of the control area: ticket, then three counter arrays of MV_CTR words.
constexpr int MV_CTR = 40;
constexpr int MV_HDR = 4 + 3 * MV_CTR;

// Exchange unit of one scanline, one step parity and one of the two searches: the plane of
// x results [QYP + 2 HB][QXP] (HB rows of PADV above and below), the column minima of each
// wavefront [NV][QXP] and the vertex minima of each wavefront [NV] (three label dimensions: the
// plane of slices [QZP + 2 HB][64] and the minima that MvTile3 lists, then the vertex minima).
template <class M, int HB>
constexpr int mv_xs() {
    return (M::PH + 2 * HB) * M::PW + M::CM + (M::NV > 4 ? M::NV : 4);
}

template <class M, int HB>
constexpr size_t mv_lds_bytes_t(int rows, int ring) {
    return ((size_t)MV_HDR + (size_t)rows * 4 * mv_xs<M, HB>() + (size_t)rows * ring * M::QT) * 4;
}

// Smallest of N consecutive LDS counters (N = 1, 2, 4, 8; 4 N-byte aligned up to 16 bytes), read
// with one access (two for N = 8).
template <int N>
__device__ __forceinline__ int32_t lds_min_ctr(const int32_t* p) {
    // an explicit LDS pointer: a generic one would become a flat access, which also counts as a
    // vector memory operation and makes waits for it wait for the prefetched loads too
    typedef __attribute__((address_space(3))) const volatile int32_t lds_i32;
    if constexpr (N == 8) {
        typedef int32_t v4 __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(3))) const volatile v4 lds_v4;
        const v4 a = *(lds_v4*)(lds_i32*)p;
        const v4 b = *(lds_v4*)(lds_i32*)(p + 4);
        return imin(imin(imin(a[0], a[1]), imin(a[2], a[3])), imin(imin(b[0], b[1]), imin(b[2], b[3])));
    } else if constexpr (N == 4) {
        typedef int32_t v4 __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(3))) const volatile v4 lds_v4;
        const v4 v = *(lds_v4*)(lds_i32*)p;
        return imin(imin(v[0], v[1]), imin(v[2], v[3]));
    } else if constexpr (N == 2) {
        typedef int32_t v2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(3))) const volatile v2 lds_v2;
        const v2 v = *(lds_v2*)(lds_i32*)p;
        return imin(v[0], v[1]);
    } else {
        return lds_get(p);
    }
}

// Minima over the four 16-lane rows of the wavefront of two values at once (every lane gets both):
// one swap halves across 32 lanes with each value in one half, the rest as in rows_min4.
__device__ __forceinline__ void rows_min4x2(int32_t& p, int32_t& q) {
    const auto a = __builtin_amdgcn_permlane32_swap(p, q, false, false);   // [p0 p1 q0 q1], [p2 p3 q2 q3]
    int32_t m = imin((int32_t)a[0], (int32_t)a[1]);                        // [p01' p13' q02' q13'] by row
    const auto b = __builtin_amdgcn_permlane16_swap(m, m, false, false);   // [m0 m0 m2 m2], [m1 m1 m3 m3]
    m = imin((int32_t)b[0], (int32_t)b[1]);                                // rows 0,1: min p; rows 2,3: min q
    const auto c = __builtin_amdgcn_permlane32_swap(m, m, false, false);   // [m0 m1 m0 m1], [m2 m3 m2 m3]
    p = (int32_t)c[0];
    q = (int32_t)c[1];
}

// Minimum over the four 16-lane rows of the wavefront (every lane gets it).
__device__ __forceinline__ int32_t rows_min4(int32_t v) {
    const auto a = __builtin_amdgcn_permlane32_swap(v, v, false, false);   // [r0 r1 r0 r1], [r2 r3 r2 r3]
    v = imin((int32_t)a[0], (int32_t)a[1]);
    const auto b = __builtin_amdgcn_permlane16_swap(v, v, false, false);   // [r0 r0 r2 r2], [r1 r1 r3 r3]
    return imin((int32_t)b[0], (int32_t)b[1]);
}

// The window candidates along x of one 16-lane row: o[k] = min over |u| <= NWK of h[k + u] + pen[u - 1]
// (h[k] itself for u = 0), the labels k + u of the row lying in this lane or the lanes to the left and
// right (a lane whose source lies outside the row keeps its value).  One asm block per label count:
// the penalised candidates are formed first and every DPP read comes at least two instructions after
// the VALU write of its source, so the block needs no wait states of its own.
#define EDP_DPP_MIN(o, p, ctl) "v_min_i32_dpp " o ", " p ", " o " " ctl " row_mask:0xf bank_mask:0xf\n\t"
template <int K, int NWK>
__device__ __forceinline__ void xwin_candidates(const int32_t (&h)[K], const int32_t (&pen)[2], int32_t (&o)[K]) {
    if constexpr (K == 1 && NWK == 1) {
        int32_t p0;
        asm volatile("v_add_u32 %1, %3, %2\n\t"
                     "v_mov_b32 %0, %2\n\t"
                     "s_nop 0\n\t"
                     EDP_DPP_MIN("%0", "%1", "row_shr:1")
                     EDP_DPP_MIN("%0", "%1", "row_shl:1")
                     : "=&v"(o[0]), "=&v"(p0) : "v"(h[0]), "s"(pen[0]));
    } else if constexpr (K == 1 && NWK == 2) {
        int32_t p0, p1;
        asm volatile("v_add_u32 %1, %4, %3\n\t"
                     "v_add_u32 %2, %5, %3\n\t"
                     "v_mov_b32 %0, %3\n\t"
                     EDP_DPP_MIN("%0", "%1", "row_shr:1")
                     EDP_DPP_MIN("%0", "%2", "row_shr:2")
                     EDP_DPP_MIN("%0", "%1", "row_shl:1")
                     EDP_DPP_MIN("%0", "%2", "row_shl:2")
                     : "=&v"(o[0]), "=&v"(p0), "=&v"(p1) : "v"(h[0]), "s"(pen[0]), "s"(pen[1]));
    } else if constexpr (K == 2 && NWK == 1) {
        int32_t p00, p01;
        // %0 o0, %1 o1, %2 p00, %3 p01, %4 h0, %5 h1, %6 pen0
        asm volatile("v_add_u32 %3, %6, %5\n\t"
                     "v_add_u32 %2, %6, %4\n\t"
                     "v_min_i32 %0, %4, %3\n\t"
                     "v_min_i32 %1, %5, %2\n\t"
                     EDP_DPP_MIN("%0", "%3", "row_shr:1")
                     EDP_DPP_MIN("%1", "%2", "row_shl:1")
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(p00), "=&v"(p01)
                     : "v"(h[0]), "v"(h[1]), "s"(pen[0]));
    } else if constexpr (K == 2 && NWK == 2) {
        int32_t p00, p01, p10, p11;
        // %0 o0, %1 o1, %2 p00, %3 p01, %4 p10, %5 p11, %6 h0, %7 h1, %8 pen0, %9 pen1
        asm volatile("v_add_u32 %3, %8, %7\n\t"
                     "v_add_u32 %4, %9, %6\n\t"
                     "v_add_u32 %2, %8, %6\n\t"
                     "v_add_u32 %5, %9, %7\n\t"
                     "v_min_i32 %0, %6, %3\n\t"
                     "v_min_i32 %1, %7, %2\n\t"
                     EDP_DPP_MIN("%0", "%3", "row_shr:1")
                     EDP_DPP_MIN("%1", "%2", "row_shl:1")
                     EDP_DPP_MIN("%0", "%4", "row_shr:1")
                     EDP_DPP_MIN("%1", "%5", "row_shr:1")
                     EDP_DPP_MIN("%0", "%4", "row_shl:1")
                     EDP_DPP_MIN("%1", "%5", "row_shl:1")
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(p00), "=&v"(p01), "=&v"(p10), "=&v"(p11)
                     : "v"(h[0]), "v"(h[1]), "s"(pen[0]), "s"(pen[1]));
    } else if constexpr (K == 4 && NWK == 1) {
        int32_t p00, p01, p02, p03;
        // %0-%3 o0-o3, %4-%7 p00-p03, %8-%11 h0-h3, %12 pen0
        asm volatile("v_add_u32 %7, %12, %11\n\t"
                     "v_add_u32 %4, %12, %8\n\t"
                     "v_add_u32 %5, %12, %9\n\t"
                     "v_add_u32 %6, %12, %10\n\t"
                     "v_min_i32 %0, %8, %5\n\t"
                     "v_min3_i32 %1, %9, %4, %6\n\t"
                     "v_min3_i32 %2, %10, %5, %7\n\t"
                     "v_min_i32 %3, %11, %6\n\t"
                     EDP_DPP_MIN("%0", "%7", "row_shr:1")
                     EDP_DPP_MIN("%3", "%4", "row_shl:1")
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]),
                       "=&v"(p00), "=&v"(p01), "=&v"(p02), "=&v"(p03)
                     : "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "s"(pen[0]));
    } else {
        static_assert(K == 4 && NWK == 2, "label counts per lane: 1, 2, 4");
        int32_t p00, p01, p02, p03, p10, p11, p12, p13;
        // %0-%3 o0-o3, %4-%7 p00-p03, %8-%11 p10-p13, %12-%15 h0-h3, %16 pen0, %17 pen1
        asm volatile("v_add_u32 %7, %16, %15\n\t"       // p03
                     "v_add_u32 %10, %17, %14\n\t"      // p12
                     "v_add_u32 %11, %17, %15\n\t"      // p13
                     "v_add_u32 %8, %17, %12\n\t"       // p10
                     "v_add_u32 %4, %16, %12\n\t"       // p00
                     "v_add_u32 %9, %17, %13\n\t"       // p11
                     "v_add_u32 %5, %16, %13\n\t"       // p01
                     "v_add_u32 %6, %16, %14\n\t"       // p02
                     "v_min3_i32 %0, %12, %5, %10\n\t"  // k0: p01, p12
                     "v_min3_i32 %1, %13, %4, %6\n\t"   // k1: p00, p02, then p13
                     "v_min3_i32 %2, %14, %5, %7\n\t"   // k2: p01, p03, then p10
                     "v_min3_i32 %3, %15, %6, %9\n\t"   // k3: p02, p11
                     "v_min_i32 %1, %1, %11\n\t"
                     "v_min_i32 %2, %2, %8\n\t"
                     EDP_DPP_MIN("%0", "%7", "row_shr:1")
                     EDP_DPP_MIN("%0", "%10", "row_shr:1")
                     EDP_DPP_MIN("%1", "%11", "row_shr:1")
                     EDP_DPP_MIN("%2", "%8", "row_shl:1")
                     EDP_DPP_MIN("%3", "%4", "row_shl:1")
                     EDP_DPP_MIN("%3", "%9", "row_shl:1")
                     : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]),
                       "=&v"(p00), "=&v"(p01), "=&v"(p02), "=&v"(p03),
                       "=&v"(p10), "=&v"(p11), "=&v"(p12), "=&v"(p13)
                     : "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "s"(pen[0]), "s"(pen[1]));
    }
}
#undef EDP_DPP_MIN

// Minimum of each of N x-lines (the lane's K labels on each 16-lane row), all N computed before
// any is used: the DPP moves of the N chains interleave (no wait states between them), and
// the last move of each chain stays in the block of its minimum, where the two fuse.
template <int K, int N>
__device__ __forceinline__ void xline_mins(const int32_t (*const (&rows)[N])[K], int32_t (&m)[N], const int32_t lane) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int32_t v = (*rows[i])[0];
#pragma unroll
        for (int k = 1; k < K; ++k) v = imin(v, (*rows[i])[k]);
        m[i] = line_min<16, 1>(v, lane);
    }
    if constexpr (N == 4) asm volatile("" : "+v"(m[0]), "+v"(m[1]), "+v"(m[2]), "+v"(m[3]));
    else if constexpr (N == 8)
        asm volatile("" : "+v"(m[0]), "+v"(m[1]), "+v"(m[2]), "+v"(m[3]), "+v"(m[4]), "+v"(m[5]), "+v"(m[6]), "+v"(m[7]));
    else
#pragma unroll
        for (int i = 0; i < N; ++i) asm volatile("" : "+v"(m[i]));
}

// Window minimum along x of the lane's K labels on one 16-lane row (one x-line per row): steps
// u = 1..NWK with penalties pen[u-1] (PEN_OFF disables a step), then the clip at the line minimum
// m + clipx.  clipx: the clip offset, or 2^30 for no clip (every value lies below line minimum +
// 2^30, and the sum stays inside int32 since values lie below PADV).
template <int K, int NWK>
__device__ __forceinline__ void xwin16(int32_t (&h)[K], const int32_t (&pen)[2], const int32_t m, const int32_t clipx) {
    int32_t o[K];
    xwin_candidates<K, NWK>(h, pen, o);
    const int32_t cap = m + clipx;
#pragma unroll
    for (int k = 0; k < K; ++k) h[k] = imin(o[k], cap);
}

// NT: the sums' loads and stores are non-temporal (the host sets it where one array of sums
// outgrows the memory-side cache, so nothing would be found there again).
template <class M, class CK, int MS, int PF, bool NT>
__global__ __launch_bounds__(64 * (MV_MAX_WAVES + 2)) void edp_pass_mv_kernel(const PassArgs a) {
    constexpr int KX = M::KX, KY = M::KY, NV = M::NV, E = M::E, QT = M::QT, QXP = M::QXP, SY = M::SY;
    constexpr int CB = CostBytes<CK>::value;
    static_assert(MS == MS_WINDOW || MS == MS_WINDOW1, "window kinds only");
    constexpr int NWK = MS == MS_WINDOW1 ? 1 : 2;    // window steps per side
    constexpr int HB = NWK;                          // halo rows of the y window
    constexpr int XS = mv_xs<M, HB>();
    constexpr int PLANE = (M::PH + 2 * HB) * M::PW;
    extern __shared__ int32_t lds[];
    int32_t* const misc = lds;                       // [0] ticket broadcast
    int32_t* const wr = lds + 4;                     // [r * NV + w] columns written into ring r
    int32_t* const rd = wr + MV_CTR;                 // [r * NV + w] columns taken from ring r
    int32_t* const xc = rd + MV_CTR;                 // [r * NV + w] steps whose exchange is written
    const int32_t RW = ((int32_t)(blockDim.x >> 6) - 2) / NV;   // scanlines; the last two wavefronts help
    int32_t* const xch = lds + MV_HDR;               // [RW][2 parity][2 search][XS]
    int32_t* const rings = xch + RW * 4 * XS;        // [RW][ring][QT]: ring r feeds scanline r

    const int32_t lane = lane_id();
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t row = wave / NV, w = wave % NV;
    const int32_t px = lane & 15, lr = lane >> 4;
    const int32_t vx0 = px * KX, vy0 = w * SY + lr * KY;
    const int32_t R = a.ring;
    const int32_t lofs = (w * 64 + lane) * E * 4;    // lane-major vertex layout

    // the halo rows of every exchange plane hold PADV for the whole launch
    for (int32_t k = threadIdx.x; k < RW * 4 * 2 * HB * M::PW; k += blockDim.x) {
        const int32_t unit = k / (2 * HB * M::PW), e = k % (2 * HB * M::PW);
        const int32_t r = e / M::PW, c = e % M::PW;
        xch[unit * XS + (r < HB ? r : M::PH + r) * M::PW + c] = PADV;
    }

    for (;;) {
        if (threadIdx.x == 0) misc[0] = (int32_t)atomicAdd(a.ticket, 1u);
        if (threadIdx.x < 3 * MV_CTR) wr[threadIdx.x] = 0;
        __syncthreads();
        const int32_t tk = __builtin_amdgcn_readfirstlane(misc[0]);
        __syncthreads();
        if (tk >= a.npass * a.tickets_per_pass) break;
        const bool second = tk >= a.tickets_per_pass;
        const int32_t rem = second ? tk - a.tickets_per_pass : tk;
        const PassDir& pd = second ? a.dir[1] : a.dir[0];
        const int32_t pass_index = pd.pass_index;
        const InstDesc d = a.ndesc > 0 ? uniform_desc(a.descs[find_instance(a.descs, a.ndesc, rem, 0)]) : a.one;
        const int32_t super = rem - d.first_ticket;
        const int32_t W = d.W, H = d.H;
        uint32_t* const done = d.flags + 2 * d.nsuper;
        if (second) {
            // start once the first scan has completed this band and the next one (see edp_pass_kernel)
            if (threadIdx.x == 0) {
                const uint32_t want = (uint32_t)a.dir[0].pass_index + 1;
                const int32_t last = super + 1 < d.nsuper ? super + 1 : super;
                for (int32_t b = super; b <= last; ++b) {
                    uint32_t spins = 0;
#pragma nounroll
                    while (flag_get(done + b) < want) {
                        if (++spins > SPIN_LIMIT_BAND || flag_get(a.error) != 0) {
                            raise_error(a.error);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const int32_t nact = min(RW, H - super * RW);      // scanlines of this band
        const bool gout = super * RW + nact < H;           // a band below takes the last scanline's T_b
        const size_t hrow = (size_t)W * QT;
        const int32_t sc = second ? 1 : 0;
        // tags (scan, band, column) are distinct within a solve (checked by the host)
        const uint32_t tag_out = ((uint32_t)pass_index * (uint32_t)d.nsuper + (uint32_t)super) * (uint32_t)(W + 1) + 1u;
        const uint32_t tag_in = tag_out - (uint32_t)(W + 1);
        if (wave >= RW * NV) {
            // Row-in helpers (two wavefronts, each the slabs sl with sl % 2 == its index): fill ring 0
            // with T_b of the band above (zeros above the first band).  Each round polls the tagged
            // words of NC columns and publishes the leading run of complete columns.  The helpers
            // run at the highest wave priority: they mostly sleep, and the compute wavefronts that
            // spin on their counters must not starve them of issue slots.
            __builtin_amdgcn_s_setprio(3);
            const int32_t hx = wave - RW * NV;             // 0 or 1
            constexpr int NS = NV / 2 > 0 ? NV / 2 : 1;    // slabs per helper
            constexpr int NC = NS * E <= 8 ? 4 : (NS * E <= 16 ? 2 : 1);   // columns per poll
            if (super == 0) {
                // zeros above the first band: each helper clears the ring words of exactly the
                // slabs whose count it publishes (slab v: 64 E words per slot from v 64 E), so a
                // slab's wavefront never reads words the other helper has not cleared yet (the
                // ring still holds the workgroup's previous band)
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v % 2 == hx)
                        for (int32_t k = lane; k < R * 64 * E; k += 64)
                            rings[(k / (64 * E)) * QT + v * 64 * E + k % (64 * E)] = 0;
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v % 2 == hx) lds_put(wr + v, W);
            } else if (hx < NV) {
                // the band above's row: [W][NV][E][64] tagged words (word k of lane l of slab w at
                // (w E + k) 64 + l, so a wavefront's access to word k is 512 contiguous bytes)
                const unsigned long long* const hrow0 = d.hand + (size_t)(sc * 2 + ((super - 1) & 1)) * hrow;
                const unsigned long long* const hin = hrow0 + lane;
                int32_t cin = 0, taken = 0;
                uint32_t spins = 0;
                bool dead = false;
#pragma nounroll
                while (cin < W && !dead) {
                    // ring space for NC columns: row 0's wavefronts of these slabs have taken cin + NC - R
                    const int32_t need = min(W, cin + NC) - R;
                    if (taken < need) {
                        int32_t t = PADV;
#pragma unroll
                        for (int i = 0; i < NS; ++i)
                            if (hx + 2 * i < NV) t = imin(t, lds_get(rd + hx + 2 * i));
                        taken = t;
                    }
                    const int32_t n = min(min(W - cin, NC), taken + R - cin);
                    int32_t got = 0;
                    if (n > 0) {
                        // probe: one word per column and slab (the slab's last word); only columns whose
                        // probes carry their tags are read in full, so polling moves a few words
                        const int32_t pc = lane / NS, pi = lane % NS;
                        const bool probe = pc < n && hx + 2 * pi < NV;
                        const unsigned long long pw =
                            probe ? tag_get(hrow0 + (size_t)(cin + pc) * QT + (size_t)((hx + 2 * pi) * E + E - 1) * 64 + 63)
                                  : 0ull;
                        const bool pok = !probe || (uint32_t)(pw >> 32) == tag_in + (uint32_t)(cin + pc);
                        const unsigned long long pm = __ballot(pok);
                        int32_t ready = 0;
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const unsigned long long cm = ((1ull << NS) - 1) << (c * NS);
                            if (ready == c && c < n && (pm & cm) == cm) ready = c + 1;
                        }
                        if (ready > 0) {
                            unsigned long long v[NC][NS][E];
#pragma unroll
                            for (int c = 0; c < NC; ++c)
#pragma unroll
                                for (int i = 0; i < NS; ++i)
#pragma unroll
                                    for (int k = 0; k < E; ++k)
                                        v[c][i][k] = (c < ready && hx + 2 * i < NV)
                                                         ? tag_get(hin + (size_t)(cin + c) * QT + ((hx + 2 * i) * E + k) * 64)
                                                         : 0ull;
                            bool run = true;
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                bool good = c < ready;
                                const uint32_t want = tag_in + (uint32_t)(cin + c);
#pragma unroll
                                for (int i = 0; i < NS; ++i)
#pragma unroll
                                    for (int k = 0; k < E; ++k)
                                        good = good && (hx + 2 * i >= NV || (uint32_t)(v[c][i][k] >> 32) == want);
                                run = run && __all(good);
                                if (run) got = c + 1;
                            }
#pragma unroll
                            for (int c = 0; c < NC; ++c) {
                                if (c < got) {
                                    int32_t* slot = rings + (size_t)((cin + c) & (R - 1)) * QT + lane * E;
#pragma unroll
                                    for (int i = 0; i < NS; ++i)
                                        if (hx + 2 * i < NV) {
#pragma unroll
                                            for (int k = 0; k < E; ++k)
                                                slot[(hx + 2 * i) * 64 * E + k] = (int32_t)(uint32_t)v[c][i][k];
                                        }
                                }
                            }
                        }
                        if (got > 0) {
                            __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
                            for (int i = 0; i < NS; ++i)
                                if (hx + 2 * i < NV) lds_put(wr + hx + 2 * i, cin + got);
                            cin += got;
                        }
                    }
                    if (got > 0) {
                        spins = 0;
                    } else {
                        if (++spins > SPIN_LIMIT || ((spins & 1023) == 0 && flag_get(a.error) != 0)) {
                            raise_error(a.error);
                            dead = true;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else if (row < nact) {
            // the band's last scanline hands its row to the next band: it goes first on its SIMDs
            // (0.3% faster side by side)
            if (row == nact - 1) __builtin_amdgcn_s_setprio(1);
            const int32_t Q = M::D3 ? d.qx * d.qy * d.qz : d.qx * d.qy;
            const int32_t sx = pd.sx, sy = pd.sy, ka = pd.ka, kb = pd.kb;
            const int32_t tbytes = W * H * QT * 4;
            int32_t* const t_b = kb == 3 ? d.t[3] : d.t[2];
            int32_t* const t_a = ka ? d.t[1] : d.t[0];
            int32_t* const t_ma = ka ? d.t[0] : d.t[1];
            int32_t* const t_mb = kb == 3 ? d.t[2] : d.t[3];
            const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(d.cost, W * H * Q * CB);
            // the last P4 forms the labels and leaves its sums unstored (nothing reads them later)
            const bool marg = pd.marginal != 0;
            const __amdgpu_buffer_rsrc_t rs_a = make_rsrc(t_a, marg ? 0 : tbytes);
            const __amdgpu_buffer_rsrc_t rs_ma = make_rsrc(t_ma, pd.old_a_zero ? 0 : tbytes);
            const __amdgpu_buffer_rsrc_t rs_mb = make_rsrc(t_mb, pd.old_b_zero ? 0 : tbytes);
            const __amdgpu_buffer_rsrc_t rs_bo = make_rsrc(t_b, pd.b_live && !marg ? tbytes : 0);
            const bool joint = d.joint != 0;
            const int32_t clipd = d.clipd;
            const int32_t clipx = joint ? 0x40000000 : clipd;   // x lines clip only per dimension
            const WinPen wp(d.lam, d.trunc, d.qx, d.qy, d.squared != 0, M::D3 ? d.qz : 1);
            int32_t crun[KY];
            bool valid[KY][KX];
            // three label dimensions: lane (px3, py3) of slab w, row ky = slice w KY + ky
            const int32_t px3 = lane & 7, py3 = lane >> 3;
            int32_t lab3[KY];                              // flat label of each slice (marginal)
            if constexpr (M::D3) {
#pragma unroll
                for (int ky = 0; ky < KY; ++ky) {
                    const int32_t vz = w * KY + ky;
                    lab3[ky] = (vz * d.qy + py3) * d.qx + px3;
                    valid[ky][0] = px3 < d.qx && py3 < d.qy && vz < d.qz;
                    crun[ky] = valid[ky][0] ? lab3[ky] * CB : OOB;
                }
            } else {
#pragma unroll
                for (int ky = 0; ky < KY; ++ky) {
                    const int32_t vy = vy0 + ky;
                    crun[ky] = (vy < d.qy && vx0 < d.qx) ? (vy * d.qx + vx0) * CB : OOB;
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) valid[ky][kx] = vx0 + kx < d.qx && vy < d.qy;
                }
            }
            // the lane holds a real label
            const bool rowok = M::D3 ? (px3 < d.qx && py3 < d.qy && w * KY < d.qz) : (vx0 < d.qx && vy0 < d.qy);
            const int32_t j = super * RW + row;             // scan-order row index
            const int32_t y = sy > 0 ? j : H - 1 - j;
            const int32_t yn = y + sy;
            const bool has_next = j + 1 < H;
            const int32_t x0 = sx > 0 ? 0 : W - 1;
            const int32_t dc = sx * Q * CB, dt = sx * QT * 4;
            const int32_t bc = cell_off(y * W + x0, Q * CB);
            const int32_t bt = cell_off(y * W + x0, QT * 4) + lofs;
            const int32_t ba = bt + dt;
            const int32_t bb = cell_off(yn * W + x0, QT * 4) + lofs;
            const int32_t nsteps = (W + PF - 1) / PF * PF;
            // labels of the row (last P4), written as global (not flat) stores: a flat store also
            // counts against the LDS wait counter, so the next LDS wait would wait for it
            gu32* const lab_row = (gu32*)(d.labels + (size_t)y * W + x0);

            // T_b of the scanline above through ring `row`; this scanline's T_b into ring row + 1 or,
            // for the band's last scanline, as tagged words for the band below
            const int32_t* const ring_in = rings + (size_t)row * R * QT + w * 64 * E + lane * E;
            const bool to_ring = row + 1 < nact;
            const bool to_mem = !to_ring && gout;
            int32_t* const ring_out = rings + (size_t)(row + 1 < RW ? row + 1 : row) * R * QT + w * 64 * E + lane * E;
            unsigned long long* const hout = d.hand + (size_t)(sc * 2 + (super & 1)) * hrow + (size_t)w * 64 * E + lane;
            int32_t* const wr_in = wr + row * NV + w;
            int32_t* const rd_in = rd + row * NV + w;
            int32_t* const wr_out = wr + (row + 1) * NV + w;
            int32_t* const rd_out = rd + (row + 1) * NV + w;
            int32_t* const xc_row = xc + row * NV;
            int32_t* const xrow = xch + row * 4 * XS;

            constexpr int CW = CostWords<CK, KX>::value;
            int32_t rc[PF][KY][CW], rma[PF][KY][KX], rmb[PF][KY][KX];
            int32_t carry[KY][KX];
#pragma unroll
            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) carry[ky][kx] = 0;
            // once a wait has given up (the error word is set, the results are void) the wavefront
            // stops waiting, so a broken schedule ends after one bounded wait per wavefront
            bool dead = false;
            auto give_up = [&](uint32_t& spins) -> bool {
                if (++spins > SPIN_LIMIT || ((spins & 1023) == 0 && flag_get(a.error) != 0)) {
                    raise_error(a.error);
                    dead = true;
                }
                return dead;
            };

            // each sum is read once, by a later scan: where the arrays outgrow the memory-side
            // cache their loads and stores are non-temporal (1.7% faster on the 961-label solve
            // 640x480; 3% slower at 320x240 with 256 labels, whose sums the cache still holds;
            // non-temporal cost loads, which the fused second scan repeats, were 2% slower)
            constexpr int SUMS_NT = NT ? 2 : 0;
            auto fetch = [&](const int32_t t, int32_t (&c)[KY][CW], int32_t (&ma)[KY][KX], int32_t (&mb)[KY][KX]) {
                const bool act = rowok && t < W;
                const int32_t offc = act ? bc + t * dc : OOB;
                const int32_t offa = (act && t + 1 < W) ? ba + t * dt : OOB;
                const int32_t offb = (act && has_next) ? bb + t * dt : OOB;
#pragma unroll
                for (int ky = 0; ky < KY; ++ky) load_cost_words<CK, KX>(rs_c, offc + crun[ky], c[ky]);
                load_vec<E, SUMS_NT>(rs_ma, offa, &ma[0][0]);
                load_vec<E, SUMS_NT>(rs_mb, offb, &mb[0][0]);
            };
#pragma unroll
            for (int u = 0; u < PF; ++u) fetch(u, rc[u], rma[u], rmb[u]);

            // T_b of the scanline above at column t, with its count: read at the end of step t - 1
            int32_t in_ready = 0, in_lb[E];
            auto read_input = [&](const int32_t t) {
                const int32_t* slot = ring_in + (size_t)(t & (R - 1)) * QT;
                in_ready = lds_get(wr_in);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
                for (int k = 0; k < E; ++k) in_lb[k] = slot[k];
            };
            read_input(0);
            int32_t taken = 0;                             // columns the next scanline has taken (lower bound)

            // CHECK: steps at or past the end of the row exist (the last round)
            auto step = [&](auto chk, const int u, const int32_t s) {
                constexpr bool CHECK = decltype(chk)::value;
                const bool live = !CHECK || s < W;         // wave-uniform
                int32_t lb[E];
#pragma unroll
                for (int k = 0; k < E; ++k) lb[k] = 0;
                if (live) {
                    uint32_t spins = 0;
                    // a waiting wavefront sleeps between polls, leaving its SIMD's issue slots to the
                    // wavefronts of the other scanlines
#pragma nounroll
                    while (in_ready < s + 1) {
                        if (dead || give_up(spins)) break;
                        __builtin_amdgcn_s_sleep(1);
                        read_input(s);
                    }
#pragma unroll
                    for (int k = 0; k < E; ++k) lb[k] = in_lb[k];
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    lds_put(rd_in, s + 1);
                }
                int32_t h[KY][KX], h2[KY][KX];
#pragma unroll
                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) {
                        const int32_t A = cost_elem<CK, KX>(rc[u][ky], kx) + carry[ky][kx] + lb[ky * KX + kx];
                        const int32_t dd = rmb[u][ky][kx] - rma[u][ky][kx];
                        h[ky][kx] = valid[ky][kx] ? ((A + dd) >> 1) : PADV;
                        h2[ky][kx] = valid[ky][kx] ? ((A - dd) >> 1) : PADV;
                    }
                // T_b leaves the wavefront (the next scanline's ring, or tagged words for the band
                // below); with two label dimensions as soon as its windows are done, ahead of T_a's
                // last window and the stores of the sums, since the next scanline waits for it
                // (2% faster on the 961-label solve)
                auto emit_b = [&]() {
                    if (live) {
                        if (to_ring) {
                            if (taken < s + 1 - R) {
                                uint32_t spins = 0;
#pragma nounroll
                                while ((taken = lds_get(rd_out)) < s + 1 - R) {
                                    if (dead || give_up(spins)) break;
                                    __builtin_amdgcn_s_sleep(1);
                                }
                            }
                            int32_t* dst = ring_out + (size_t)(s & (R - 1)) * QT;
#pragma unroll
                            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                                for (int kx = 0; kx < KX; ++kx) dst[ky * KX + kx] = h2[ky][kx];
                            __atomic_signal_fence(__ATOMIC_SEQ_CST);
                            lds_put(wr_out, s + 1);
                        } else if (to_mem) {
                            const unsigned long long tg = (unsigned long long)(tag_out + (uint32_t)s) << 32;
#pragma unroll
                            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                                for (int kx = 0; kx < KX; ++kx)
                                    tag_put(hout + (size_t)s * QT + (ky * KX + kx) * 64, tg | (uint32_t)h2[ky][kx]);
                        }
                    }
                };
                if constexpr (M::D3) {
                    // ---- windows along x and y inside the wavefront (each of its slices), both sums
                    const int32_t g1 = min_search_xy<typename M::Lane, NWK>(h, wp, clipd, joint, lane);
                    const int32_t g2 = min_search_xy<typename M::Lane, NWK>(h2, wp, clipd, joint, lane);
                    const int32_t par = s & 1;
                    int32_t* const u1 = xrow + (par * 2 + 0) * XS;
                    int32_t* const u2 = xrow + (par * 2 + 1) * XS;
                    if (marg) {
                        // marginal of eq. DP_2D_1 at this vertex (as for two label dimensions)
                        int32_t bv = 0x7FFFFFFF, bl = 0x7FFFFFFF;
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky) {
                            const int32_t A = cost_elem<CK, KX>(rc[u][ky], 0) + carry[ky][0] + lb[ky];
                            const int32_t v = A + rma[u][ky][0] + rmb[u][ky][0];
                            const bool better = valid[ky][0] && v < bv;   // labels rise with ky
                            bv = better ? v : bv;
                            bl = better ? lab3[ky] : bl;
                        }
                        const int32_t wv = rows_min4(line_min<16, 1>(bv, lane));
                        const int32_t wl = rows_min4(line_min<16, 1>(bv == wv ? bl : 0x7FFFFFFF, lane));
                        if (lane == 0) {
                            u1[PLANE + M::CM + w] = wv;
                            u2[PLANE + M::CM + w] = wl;
                        }
                    }
                    // ---- exchange: the wavefront's slices, its per-lane minimum over them (the
                    // clip of the z-lines) and its minimum over all its labels (the joint clip)
                    int32_t m1 = h[0][0], m2 = h2[0][0];
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky) {
                        u1[(HB + w * KY + ky) * 64 + lane] = h[ky][0];
                        u2[(HB + w * KY + ky) * 64 + lane] = h2[ky][0];
                        m1 = imin(m1, h[ky][0]);
                        m2 = imin(m2, h2[ky][0]);
                    }
                    u1[PLANE + w * 64 + lane] = m1;
                    u2[PLANE + w * 64 + lane] = m2;
                    if (lane == 0) {
                        u1[PLANE + NV * 64 + w] = g1;
                        u2[PLANE + NV * 64 + w] = g2;
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    lds_put(xc_row + w, s + 1);
                    {
                        uint32_t spins = 0;
#pragma nounroll
                        while (lds_min_ctr<NV>(xc_row) < s + 1) {
                            if (dead || give_up(spins)) break;
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (marg && w == 0) {
                        int32_t fv = u1[PLANE + M::CM], fl = u2[PLANE + M::CM];
#pragma unroll
                        for (int v = 1; v < NV; ++v) {
                            const int32_t ov = u1[PLANE + M::CM + v], ol = u2[PLANE + M::CM + v];
                            fl = ov < fv ? ol : (ov == fv ? imin(fl, ol) : fl);
                            fv = imin(fv, ov);
                        }
                        if (lane == 0 && live) lab_row[sx * s] = (uint32_t)fl;
                    }
                    // ---- window along z: own slices plus HB slices below and above; clip at the
                    // z-line minimum (per-dimension truncation), or at the vertex minimum after the
                    // window (joint truncation)
#pragma unroll
                    for (int srch = 0; srch < 2; ++srch) {
                        int32_t (&hv)[KY][KX] = srch ? h2 : h;
                        const int32_t* const un = srch ? u2 : u1;
                        const int32_t* const ez = un + w * KY * 64 + lane;   // slices w KY - HB ..
                        int32_t e[KY + 2 * HB];
#pragma unroll
                        for (int i = 0; i < KY + 2 * HB; ++i) e[i] = ez[i * 64];
                        int32_t cap = 0x7FFFFFFF;
                        if (!joint) {
                            int32_t zm = un[PLANE + lane];
#pragma unroll
                            for (int v = 1; v < NV; ++v) zm = imin(zm, un[PLANE + v * 64 + lane]);
                            cap = zm + clipd;
                        }
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky) {
                            int32_t o = imin(e[HB + ky], cap);
#pragma unroll
                            for (int st = 1; st <= NWK; ++st)
                                o = imin3(o, e[HB + ky - st] + wp.pz[st - 1], e[HB + ky + st] + wp.pz[st - 1]);
                            hv[ky][0] = o;
                        }
                        if (joint) {
                            int32_t g = un[PLANE + NV * 64];
#pragma unroll
                            for (int v = 1; v < NV; ++v) g = imin(g, un[PLANE + NV * 64 + v]);
#pragma unroll
                            for (int ky = 0; ky < KY; ++ky) hv[ky][0] = imin(hv[ky][0], g + clipd);
                        }
                    }
                } else {
                    // ---- window along x (lane rows), both sums
                    int32_t xm[2 * KY];
                    {
                        const int32_t (*rows[2 * KY])[KX];
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky) {
                            rows[2 * ky] = &h[ky];
                            rows[2 * ky + 1] = &h2[ky];
                        }
                        xline_mins<KX, 2 * KY>(rows, xm, lane);
                    }
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky) {
                        xwin16<KX, NWK>(h[ky], wp.px, xm[2 * ky], clipx);
                        xwin16<KX, NWK>(h2[ky], wp.px, xm[2 * ky + 1], clipx);
                    }
                    // ---- exchange: label rows next to the lane rows' edges, column minima per wavefront
                    const int32_t par = s & 1;
                    int32_t* const u1 = xrow + (par * 2 + 0) * XS;
                    int32_t* const u2 = xrow + (par * 2 + 1) * XS;
                    if (marg) {
                        // marginal of eq. DP_2D_1 at this vertex: C + T_-x(x + 1) + T_-y(y + 1) (this scan's
                        // own sums) + T_+x(x - 1) + T_+y(y - 1) (the sums it reads), so A + both old sums;
                        // this wavefront's smallest value and, among the labels holding it, the smallest label
                        int32_t bv = 0x7FFFFFFF, bl = 0x7FFFFFFF;
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                            for (int kx = 0; kx < KX; ++kx) {
                                const int32_t A = cost_elem<CK, KX>(rc[u][ky], kx) + carry[ky][kx] + lb[ky * KX + kx];
                                const int32_t v = A + rma[u][ky][kx] + rmb[u][ky][kx];
                                const bool better = valid[ky][kx] && v < bv;   // labels rise with (ky, kx)
                                bv = better ? v : bv;
                                bl = better ? (vy0 + ky) * d.qx + vx0 + kx : bl;
                            }
                        const int32_t wv = rows_min4(line_min<16, 1>(bv, lane));
                        const int32_t wl = rows_min4(line_min<16, 1>(bv == wv ? bl : 0x7FFFFFFF, lane));
                        if (lane == 0) {
                            u1[PLANE + NV * QXP + w] = wv;
                            u2[PLANE + NV * QXP + w] = wl;
                        }
                    }
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky) {
                        if (ky < HB || ky >= KY - HB) {
                            const int32_t o = (HB + vy0 + ky) * QXP + vx0;
#pragma unroll
                            for (int kx = 0; kx < KX; ++kx) {
                                u1[o + kx] = h[ky][kx];
                                u2[o + kx] = h2[ky][kx];
                            }
                        }
                    }
                    int32_t c1[KX], c2[KX];
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) {
                        c1[kx] = h[0][kx];
                        c2[kx] = h2[0][kx];
#pragma unroll
                        for (int ky = 1; ky < KY; ++ky) {
                            c1[kx] = imin(c1[kx], h[ky][kx]);
                            c2[kx] = imin(c2[kx], h2[ky][kx]);
                        }
                        rows_min4x2(c1[kx], c2[kx]);
                    }
                    // every lane row holds the same minima: all write them (no branch)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) {
                        u1[PLANE + w * QXP + vx0 + kx] = c1[kx];
                        u2[PLANE + w * QXP + vx0 + kx] = c2[kx];
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    lds_put(xc_row + w, s + 1);
                    {
                        uint32_t spins = 0;
#pragma nounroll
                        while (lds_min_ctr<NV>(xc_row) < s + 1) {
                            if (dead || give_up(spins)) break;
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (marg && w == 0) {
                        int32_t fv = u1[PLANE + NV * QXP], fl = u2[PLANE + NV * QXP];
#pragma unroll
                        for (int v = 1; v < NV; ++v) {
                            const int32_t ov = u1[PLANE + NV * QXP + v], ol = u2[PLANE + NV * QXP + v];
                            fl = ov < fv ? ol : (ov == fv ? imin(fl, ol) : fl);
                            fv = imin(fv, ov);
                        }
                        if (lane == 0 && live) lab_row[sx * s] = (uint32_t)fl;
                    }
                    // ---- window along y: own rows plus HB rows above and below; clip at the column
                    // minimum (per-dimension truncation) or at the vertex minimum (joint truncation)
#pragma unroll
                    for (int srch = 0; srch < 2; ++srch) {
                        // T_b first: it leaves the wavefront (ring or tagged words), T_a only feeds
                        // this scanline's next step
                        int32_t (&hv)[KY][KX] = srch ? h : h2;
                        const int32_t* const un = srch ? u1 : u2;
                        int32_t cmin[KX];
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx) {
                            int32_t m = un[PLANE + vx0 + kx];
#pragma unroll
                            for (int v = 1; v < NV; ++v) m = imin(m, un[PLANE + v * QXP + vx0 + kx]);
                            cmin[kx] = m;
                        }
                        // the vertex minimum of the sums equals the minimum of the x results (their
                        // window includes the label itself, with no clip in joint mode)
                        int32_t g = cmin[0];
                        if (joint) {
#pragma unroll
                            for (int kx = 1; kx < KX; ++kx) g = imin(g, cmin[kx]);
                            g = line_min<16, 1>(g, lane);
                        }
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx) {
                            int32_t e[KY + 2 * HB];
#pragma unroll
                            for (int k = 0; k < HB; ++k) {
                                e[k] = un[(vy0 + k) * QXP + vx0 + kx];                  // row vy0 - HB + k
                                e[HB + KY + k] = un[(HB + vy0 + KY + k) * QXP + vx0 + kx];   // row vy0 + KY + k
                            }
#pragma unroll
                            for (int ky = 0; ky < KY; ++ky) e[HB + ky] = hv[ky][kx];
                            const int32_t cap = (joint ? g : cmin[kx]) + clipd;
#pragma unroll
                            for (int ky = 0; ky < KY; ++ky) {
                                int32_t o = imin(e[HB + ky], cap);
#pragma unroll
                                for (int st = 1; st <= NWK; ++st)
                                    o = imin3(o, e[HB + ky - st] + wp.py[st - 1], e[HB + ky + st] + wp.py[st - 1]);
                                hv[ky][kx] = o;
                            }
                        }
                        if (srch == 0) emit_b();
                    }
                }
                // ---- outputs: T_a feeds the next vertex, T_b the next scanline
                const int32_t o = bt + s * dt;
                const bool act = rowok && live;
                store_vec<E, SUMS_NT>(rs_a, act ? o : OOB, &h[0][0]);
                store_vec<E, SUMS_NT>(rs_bo, act ? o : OOB, &h2[0][0]);
#pragma unroll
                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) carry[ky][kx] = h[ky][kx];
                if constexpr (M::D3) emit_b();   // after the stores here (measured faster)
                if (!CHECK || s + 1 < W) read_input(s + 1);
                fetch(s + PF, rc[u], rma[u], rmb[u]);
            };
            int32_t s0 = 0;
            for (; s0 + PF < W; s0 += PF) {
#pragma unroll
                for (int u = 0; u < PF; ++u) step(std::false_type{}, u, s0 + u);
            }
            for (; s0 < nsteps; s0 += PF) {
#pragma unroll
                for (int u = 0; u < PF; ++u) step(std::true_type{}, u, s0 + u);
            }
        }
        __builtin_amdgcn_s_setprio(0);
        // band complete (see edp_pass_kernel)
        if (a.npass > 1 && !second) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (a.npass > 1 && !second && threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            flag_put(done + super, (uint32_t)pass_index + 1);
        }
    }
}

// Marginal of eq. DP_2D_1 and its smallest argmin for the wide vertices: one wavefront per
// vertex, each lane the same labels as in the scans (NV slabs of E labels).
template <class M, class CT>
__global__ __launch_bounds__(256) void edp_aggregate_mv_kernel(const AggArgs a) {
    constexpr int KX = M::KX, KY = M::KY, NV = M::NV, E = M::E, QT = M::QT, SY = M::SY;
    const int32_t lane = lane_id();
    const int32_t px = lane & 15, lr = lane >> 4;
    const int32_t blk = (int32_t)blockIdx.x;
    const InstDesc d = a.ndesc > 0 ? uniform_desc(a.descs[find_instance(a.descs, a.ndesc, blk, 1)]) : a.one;
    const int32_t W = d.W, H = d.H, Q = d.qx * d.qy;
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t cells = W * H;
    if (threadIdx.x == 0 && blk == d.first_block && d.status)
        *d.status = (a.error && *a.error != 0) ? STATUS_TIMEOUT : 0;
    const int32_t cell = (blk - d.first_block) * a.cells_per_block + wave;
    const bool ok = cell < cells;
    const int32_t y = ok ? cell / W : 0, x = ok ? cell % W : 0;
    const int32_t tbytes = W * H * QT * 4;
    const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(d.cost, cells * Q * (int32_t)sizeof(CT));
    const int32_t vx0 = px * KX;
    const int32_t nb[4] = {ok && x > 0 ? cell - 1 : -1, ok && x + 1 < W ? cell + 1 : -1,
                           ok && y > 0 ? cell - W : -1, ok && y + 1 < H ? cell + W : -1};
    int32_t best = 0x7FFFFFFF, bq = 0x7FFFFFFF;
#pragma unroll
    for (int w = 0; w < NV; ++w) {
        const int32_t vy0 = w * SY + lr * KY;
        const bool live = ok && vx0 < d.qx && vy0 < d.qy;
        int32_t acc[KY][KX], tv[KY][KX];
#pragma unroll
        for (int ky = 0; ky < KY; ++ky) {
            const int32_t vy = vy0 + ky;
            const int32_t crun = (live && vy < d.qy) ? (cell * Q + vy * d.qx + vx0) * (int32_t)sizeof(CT) : OOB;
            int32_t cw[KX];
            load_cost_words<CT, KX>(rs_c, crun, cw);
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) acc[ky][kx] = cw[kx];
        }
        const int32_t lofs = (w * 64 + lane) * E * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            load_vec<E>(make_rsrc(d.t[k], tbytes), live && nb[k] >= 0 ? nb[k] * QT * 4 + lofs : OOB, &tv[0][0]);
#pragma unroll
            for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) acc[ky][kx] += tv[ky][kx];
        }
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) {
                const int32_t vy = vy0 + ky, vx = vx0 + kx;
                const int32_t lab = vy * d.qx + vx;
                const int32_t v = acc[ky][kx];
                if (live && vx < d.qx && vy < d.qy && (v < best || (v == best && lab < bq))) {
                    best = v;
                    bq = lab;
                }
            }
    }
    // smallest value, then the smallest label among the lanes holding it
    int32_t vmin = best;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) vmin = imin(vmin, __shfl_xor(vmin, sh));
    int32_t qmin = best == vmin ? bq : 0x7FFFFFFF;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) qmin = imin(qmin, __shfl_xor(qmin, sh));
    if (ok && lane == 0) d.labels[cell] = qmin;
}

}  // namespace edp
