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
// (x, y - sy): a 2D wavefront, pipelined at three levels.
//  * Lanes: a vertex takes SPLIT * G lanes.  With SPLIT = 2 the lower G lanes
//    compute T_a and the upper G lanes T_b, each with one minimum search, and
//    they exchange T_a / T_b through cross-row permutes every step.
//  * Wavefront: 64 / (SPLIT * G) scanlines run one column apart; the T_b a
//    scanline produces at step s reaches the scanline below at step s + 1.
//  * Workgroup: its wavefronts take consecutive bands of scanlines; the last
//    scanline of a band hands T_b to the next wavefront through an LDS ring
//    (progress counters in LDS).  Workgroups take whole groups of bands in
//    scan order from a ticket counter, so the group a workgroup waits on is
//    always held by a running workgroup; the last band publishes its progress
//    every `chunk` columns (release at agent scope) and the next workgroup
//    reads it from memory after an acquire.
// T_b written by P1 and P3 is only read inside the scan, so it reaches memory
// only at workgroup boundaries.  Operands that do not depend on the scan (C
// and the two "old" arrays) are prefetched PF steps ahead in a register ring.
#include "edp_device.hpp"
#include "edp_internal.hpp"

namespace edp {

constexpr int MAX_WAVES = 8;
// s_waitcnt vmcnt(0) with the other counters left open (gfx9 encoding: expcnt 7, lgkmcnt 15)
constexpr int WAIT_VMCNT0 = 0x0F70;

// Progress counters in LDS.  Every lane reads / writes the same word; the LDS
// operations of one wavefront are performed in issue order, which orders a
// counter against the ring slot written or read before it.
__device__ __forceinline__ int32_t lds_get(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_put(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// byte offset of a vertex (wrapping arithmetic: lanes off the grid discard it)
__device__ __forceinline__ int32_t cell_off(int32_t cell, int32_t bytes) {
    return (int32_t)((uint32_t)cell * (uint32_t)bytes);
}
// Flags and the error word are read and written as global (not flat) atomics:
// flat accesses may complete out of order with the buffer loads of the
// prefetch ring, which would force the compiler to drain every load in flight
// wherever a prefetched value is used.
typedef __attribute__((address_space(1))) uint32_t gu32;
__device__ __forceinline__ gu32* glob(uint32_t* p) { return (gu32*)p; }
__device__ __forceinline__ uint32_t flag_get(uint32_t* p) {
    return __hip_atomic_load(glob(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_put(uint32_t* p, uint32_t v) {
    __hip_atomic_store(glob(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void raise_error(uint32_t* error) { flag_put(error, 1u); }

// WIN: the label-window solve.  Every vertex holds an 8 x 8 frame of labels around its own
// window (costs outside the window are large), d.aux holds the frame shifts towards the four
// neighbours, and each sum handed on is evaluated in the receiving vertex's frame.
template <class T, class CK, int SPLIT, int PF, bool WIN = false>
__global__ __launch_bounds__(64 * MAX_WAVES) void edp_pass_kernel(const PassArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, E = T::E, QT = T::QT;
    constexpr int CL = SPLIT * G;                  // lanes per vertex
    constexpr int RPW = 64 / CL;                   // scanlines per wavefront
    constexpr int CB = CostBytes<CK>::value;
    static_assert(CL <= 64, "vertex wider than a wavefront");
    extern __shared__ int32_t lds[];
    int32_t* prod = lds;                           // [MAX_WAVES] columns handed to the next wavefront
    int32_t* cons = lds + MAX_WAVES;               // [MAX_WAVES] columns taken from the previous one
    int32_t* misc = lds + 2 * MAX_WAVES;           // [0] ticket broadcast
    int32_t* trash = lds + 2 * MAX_WAVES + 4;      // [QT] sink of the lanes that hand nothing over
    int32_t* rings = trash + QT;                   // [NW-1][ring][QT]
    static_assert(!WIN || SPLIT == 1, "the window solve runs both searches on every lane");

    const int32_t lane = lane_id();
    // wavefront-uniform values live in scalar registers, so control flow on them is scalar
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t NW = (int32_t)(blockDim.x >> 6);
    const int32_t grp = lane / CL;
    const bool beta = SPLIT == 2 && ((lane / G) & 1);
    const int32_t l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t R = a.ring;
    // T arrays are lane-major inside a vertex: the lane's E labels are contiguous
    const int32_t lofs = l * E * 4;

    for (;;) {
        if (threadIdx.x == 0) misc[0] = (int32_t)atomicAdd(a.ticket, 1u);
        if (threadIdx.x < 2 * MAX_WAVES) lds[threadIdx.x] = 0;
        __syncthreads();
        const int32_t tk = __builtin_amdgcn_readfirstlane(misc[0]);
        __syncthreads();
        if (tk >= a.npass * a.tickets_per_pass) break;
        // which scan of the launch, which instance, which workgroup band
        const bool second = tk >= a.tickets_per_pass;
        const int32_t rem = second ? tk - a.tickets_per_pass : tk;
        const int32_t sx = second ? a.dir[1].sx : a.dir[0].sx;
        const int32_t sy = second ? a.dir[1].sy : a.dir[0].sy;
        const int32_t ka = second ? a.dir[1].ka : a.dir[0].ka;
        const int32_t kb = second ? a.dir[1].kb : a.dir[0].kb;
        const bool old_a_zero = (second ? a.dir[1].old_a_zero : a.dir[0].old_a_zero) != 0;
        const bool old_b_zero = (second ? a.dir[1].old_b_zero : a.dir[0].old_b_zero) != 0;
        const bool b_live = (second ? a.dir[1].b_live : a.dir[0].b_live) != 0;
        const int32_t pass_index = second ? a.dir[1].pass_index : a.dir[0].pass_index;
        const InstDesc d = a.ndesc > 0 ? uniform_desc(a.descs[find_instance(a.descs, a.ndesc, rem, 0)]) : a.one;
        const int32_t super = rem - d.first_ticket;
        const int32_t W = d.W, H = d.H, Q = d.qx * d.qy;
        uint32_t* const progress = d.flags + (second ? d.nsuper : 0);
        uint32_t* const done = d.flags + 2 * d.nsuper;
        const uint32_t epoch = (uint32_t)pass_index * (uint32_t)(W + 1);
        if (second) {
            // The first scan reads, at its rows, the arrays this scan writes, and writes the
            // array this scan reads along x; both sweep the rows in the same order.  Start
            // once the first scan has completed this band and the next one (which holds the
            // row after the band's last).
            if (threadIdx.x == 0) {
                const uint32_t want = (uint32_t)a.dir[0].pass_index + 1;
                const int32_t last = super + 1 < d.nsuper ? super + 1 : super;
                for (int32_t b = super; b <= last; ++b) {
                    uint32_t spins = 0;
#pragma nounroll
                    while (flag_get(done + b) < want) {
                        if (++spins > SPIN_LIMIT_BAND ||
                            flag_get(a.error) != 0) {
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
        const bool joint = d.joint != 0;
        const LineIndex<T> li(d.lam, lane);
        // Buffer resources: a lane whose operand does not exist uses offset OOB, so
        // its load returns 0 and its store is dropped, with no branch around it.
        const int32_t tbytes = W * H * QT * 4;         // below 2^31 (checked by the host)
        const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(d.cost, W * H * Q * CB);
        // ka is 0 or 1 and kb 2 or 3: pick the arrays with selects (no indexed private array)
        int32_t* const t_a = ka ? d.t[1] : d.t[0];
        int32_t* const t_ma = ka ? d.t[0] : d.t[1];
        int32_t* const t_b = kb == 3 ? d.t[3] : d.t[2];
        int32_t* const t_mb = kb == 3 ? d.t[2] : d.t[3];
        const __amdgpu_buffer_rsrc_t rs_a = make_rsrc(t_a, tbytes);
        const __amdgpu_buffer_rsrc_t rs_b = make_rsrc(t_b, tbytes);
        const __amdgpu_buffer_rsrc_t rs_ma = make_rsrc(t_ma, tbytes);
        const __amdgpu_buffer_rsrc_t rs_mb = make_rsrc(t_mb, tbytes);
        int32_t crun[KY];                              // cost byte offset of the lane's run of KX labels
        bool valid[KY][KX];
#pragma unroll
        for (int ky = 0; ky < KY; ++ky) {
            const int32_t vy = py * KY + ky;
            crun[ky] = (vy < d.qy && px * KX < d.qx) ? (vy * d.qx + px * KX) * CB : OOB;
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) valid[ky][kx] = px * KX + kx < d.qx && vy < d.qy;
        }
        const int32_t band = super * NW + wave;
        if (band < d.nbands) {
            const int32_t j = band * RPW + grp;            // scan-order row index
            const bool rowok = j < H;
            const int32_t y = sy > 0 ? j : H - 1 - j;
            const int32_t yp = y - sy;                     // previous row in scan order
            const int32_t yn = y + sy;                     // next row in scan order
            const bool has_next = j + 1 < H;
            // Roles.  Group 0 takes the row above from memory (the first wavefront of a
            // workgroup; there is none above the first band of the scan) or from LDS (the other
            // wavefronts).  The band's last scanline goes to LDS (the next wavefront) or to
            // memory (the next workgroup, or nobody after the last band).  Each of the four
            // combinations has its own copy of the step loop, so no step branches on a role.
            const bool in_global = wave == 0;
            const bool gin = super > 0;                    // a workgroup band above exists
            const bool out_lds = wave + 1 < NW && band + 1 < d.nbands;
            const bool gout = band + 1 < d.nbands;         // a band below exists
            const bool store_a = SPLIT == 1 || !beta;
            const bool hands = grp == RPW - 1 && (SPLIT == 1 || beta);
            const int32_t* ring_in = rings + (size_t)(wave > 0 ? wave - 1 : 0) * R * QT + l;
            int32_t* ring_out = rings + (size_t)wave * R * QT + l;
            // byte offsets at step 0 (column -grp) and per-step strides: at step t the lane's
            // vertex is x = x0 + sx (t - grp) of row y
            const int32_t x0 = (sx > 0 ? 0 : W - 1) - sx * grp;
            const int32_t dc = sx * Q * CB, dt = sx * QT * 4;
            const int32_t bc = cell_off(y * W + x0, Q * CB);
            const int32_t bt = cell_off(y * W + x0, QT * 4) + lofs;
            const int32_t ba = bt + dt;                    // (x + sx, y)
            const int32_t bb = cell_off(yn * W + x0, QT * 4) + lofs;
            const int32_t bg = cell_off(yp * W + x0, QT * 4) + lofs;
            // window solve: frame-shift codes of the vertex (8 bytes per vertex)
            const int32_t bsh = cell_off(y * W + x0, 8), dsh = sx * 8;
            const __amdgpu_buffer_rsrc_t rs_sh = make_rsrc(d.aux, WIN ? W * H * 8 : 0);
            int32_t* const wscr = rings + (size_t)(NW > 1 ? NW - 1 : 0) * R * QT +
                                  (size_t)wave * 2 * 64 * (KX > KY ? KX : KY);
            // steps rounded up to whole prefetch rounds: the extra steps touch nothing (every lane
            // is past the end of its row), and a fixed count of loads per step lets the compiler
            // wait for exactly the slot in use instead of for every load in flight
            const int32_t nsteps = (W + RPW - 1 + PF - 1) / PF * PF;

            auto run = [&](auto in_tag, auto out_tag) {
                constexpr bool IG = decltype(in_tag)::value;    // row above from memory
                constexpr bool OG = decltype(out_tag)::value;   // last scanline to memory
                // T_b of the last scanline of a band that feeds a workgroup is stored coherent
                // at device scope, so the consumer needs no cache write-back or invalidation
                const bool store_b = (SPLIT == 1 || beta) && (b_live || (OG && gout && grp == RPW - 1));
                uint32_t seen = gin ? 0u : (uint32_t)W;       // columns published by the workgroup above
                int32_t taken = 0;                             // columns the next wavefront has taken (lower bound)

                constexpr int CW = CostWords<CK, KX>::value;
                int32_t rc[PF][KY][CW], rma[PF][KY][KX], rmb[PF][KY][KX], rb[PF][KY][KX];
                int32_t rsh[PF][WIN ? 2 : 1];
                int32_t carry[KY][KX], out[KY][KX];
#pragma unroll
                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) carry[ky][kx] = out[ky][kx] = rb[0][ky][kx] = 0;

                // Issue the loads of step t into one ring slot (no branch around a load).
                auto fetch = [&](const int32_t t, int32_t (&c)[KY][CW], int32_t (&ma)[KY][KX],
                                 int32_t (&mb)[KY][KX], int32_t (&gb)[KY][KX], int32_t (&sh)[WIN ? 2 : 1]) {
                    if constexpr (IG) {
                        if (t < W && seen < (uint32_t)t + 1) {       // wave-uniform
                            const uint32_t need = (uint32_t)t + 1;
                            uint32_t v = 0, spins = 0;
#pragma nounroll
                            for (;;) {
                                v = flag_get(progress + super - 1);
                                v = __builtin_amdgcn_readfirstlane(v);
                                if (v >= epoch + need) break;
                                // give up (and let every other waiter give up) instead of hanging
                                if (++spins > SPIN_LIMIT ||
                                    flag_get(a.error) != 0) {
                                    raise_error(a.error);
                                    v = epoch + (uint32_t)W;
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                            }
                            seen = v - epoch;
                            // the row is read with device-scope loads issued after this point
                            __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        }
                    }
                    // column i = t - grp of this lane's scanline; offsets move by a fixed stride per step
                    const uint32_t i = (uint32_t)(t - grp);
                    const bool act = rowok && i < (uint32_t)W;
                    const bool nxt = i + 1 < (uint32_t)W;     // the next column in scan order exists
                    const int32_t offc = act ? bc + t * dc : OOB;
                    const int32_t offa = (act && nxt && !old_a_zero) ? ba + t * dt : OOB;
                    const int32_t offb = (act && has_next && !old_b_zero) ? bb + t * dt : OOB;
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky) load_cost_words<CK, KX>(rs_c, offc + crun[ky], c[ky]);
                    load_vec<E>(rs_ma, offa, &ma[0][0]);
                    load_vec<E>(rs_mb, offb, &mb[0][0]);
                    if constexpr (IG) {
                        const int32_t offg = (act && gin && grp == 0) ? bg + t * dt : OOB;
                        load_vec<E, CPOL_DEVICE>(rs_b, offg, &gb[0][0]);
                    }
                    if constexpr (WIN) load_vec<2>(rs_sh, act ? bsh + t * dsh : OOB, sh);
                };

#pragma unroll
                for (int u = 0; u < PF; ++u) fetch(u, rc[u], rma[u], rmb[u], rb[u], rsh[u]);

                // Input of an inner wavefront: the producer's counter and the ring slot of column
                // t, read back to back.  LDS performs the operations of the CU in arrival order and
                // the producer writes a slot before the counter, so when the counter shows column t
                // the slot read issued after it returns that column.  Column t + 1 is read at the
                // end of step t, which keeps the LDS round trip off the step when the producer is
                // ahead.
                int32_t in_ready = 0, in_lb[KY][KX];
                auto read_input = [&](const int32_t t) {
                    const int32_t* slot = ring_in + (size_t)(t & (R - 1)) * QT;
                    in_ready = lds_get(prod + wave - 1);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
                    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx)
                            in_lb[ky][kx] = __hip_atomic_load(slot + (ky * KX + kx) * G, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                };
                if constexpr (!IG) read_input(0);

                for (int32_t s0 = 0; s0 < nsteps; s0 += PF) {
#pragma unroll
                    for (int u = 0; u < PF; ++u) {
                        const int32_t s = s0 + u;
                        const int32_t i = s - grp;
                        const bool act = rowok && (uint32_t)i < (uint32_t)W;
                        // T_b of the row above at this column, for group 0 of an inner wavefront
                        int32_t lb[KY][KX];
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                            for (int kx = 0; kx < KX; ++kx) lb[ky][kx] = 0;
                        if constexpr (!IG) {
                            if (s < W) {                                 // wave-uniform
                                uint32_t spins = 0;
#pragma nounroll
                                while (in_ready < s + 1) {
                                    if (++spins > SPIN_LIMIT) {
                                        raise_error(a.error);
                                        break;
                                    }
                                    read_input(s);
                                }
#pragma unroll
                                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                                    for (int kx = 0; kx < KX; ++kx) lb[ky][kx] = in_lb[ky][kx];
                                // LDS operations of a wavefront complete in order: the slot is
                                // read before the counter that frees it is written
                                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                                lds_put(cons + wave, s + 1);
                            }
                        }
                        int32_t h[KY][KX], h2[KY][KX];
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                            for (int kx = 0; kx < KX; ++kx) {
                                const int32_t v = out[ky][kx];
                                int32_t cr, mb;
                                if constexpr (SPLIT == 1) {
                                    cr = carry[ky][kx];
                                    mb = 0;
                                    if constexpr (RPW > 1) mb = lanes_up<(RPW > 1 ? CL : 1)>(v, lane);
                                } else {
                                    const int32_t x1 = lanes_up<G>(v, lane);
                                    int32_t x2 = 0;
                                    if constexpr (RPW > 1) x2 = lanes_up<(RPW > 1 ? 2 * G : 1)>(v, lane);
                                    cr = beta ? x1 : v;
                                    mb = beta ? x2 : x1;
                                    if (i == 0) cr = 0;
                                }
                                if (grp == 0) mb = IG ? rb[u][ky][kx] : lb[ky][kx];
                                const int32_t A = cost_elem<CK, KX>(rc[u][ky], kx) + cr + mb;
                                const int32_t d = rmb[u][ky][kx] - rma[u][ky][kx];
                                if constexpr (SPLIT == 1) {
                                    h[ky][kx] = valid[ky][kx] ? ((A + d) >> 1) : PADV;
                                    h2[ky][kx] = valid[ky][kx] ? ((A - d) >> 1) : PADV;
                                } else {
                                    h[ky][kx] = valid[ky][kx] ? ((A + (beta ? -d : d)) >> 1) : PADV;
                                }
                            }
                        if constexpr (WIN) {
                            // shift codes: bytes (dx, dy) towards +x, -x (dword 0) and +y, -y (dword 1)
                            const int32_t ca = rsh[u][0] >> (sx > 0 ? 0 : 16);
                            const int32_t cb = rsh[u][1] >> (sy > 0 ? 0 : 16);
                            const int32_t dxa = (int32_t)(int8_t)(ca & 0xFF), dya = (int32_t)(int8_t)((ca >> 8) & 0xFF);
                            const int32_t dxb = (int32_t)(int8_t)(cb & 0xFF), dyb = (int32_t)(int8_t)((cb >> 8) & 0xFF);
                            min_search_shift<T>(h, d.lam, d.clipd, joint, lane, dxa, dya, wscr);
                            min_search_shift<T>(h2, d.lam, d.clipd, joint, lane, dxb, dyb, wscr);
                        } else {
                            min_search<T>(h, li, d.clipd, joint, lane);
                            if constexpr (SPLIT == 1) min_search<T>(h2, li, d.clipd, joint, lane);
                        }
                        const int32_t o = bt + s * dt;
                        const int32_t oa = (act && store_a) ? o : OOB;
                        const int32_t ob = (act && store_b) ? o : OOB;
                        int32_t tbv[KY][KX];
#pragma unroll
                        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                            for (int kx = 0; kx < KX; ++kx) {
                                tbv[ky][kx] = SPLIT == 1 ? h2[ky][kx] : h[ky][kx];
                                if constexpr (SPLIT == 1) carry[ky][kx] = act ? h[ky][kx] : carry[ky][kx];
                                out[ky][kx] = tbv[ky][kx];
                            }
                        store_vec<E>(rs_a, oa, &h[0][0]);
                        if constexpr (OG) store_vec<E, CPOL_DEVICE>(rs_b, ob, &tbv[0][0]);
                        else store_vec<E>(rs_b, ob, &tbv[0][0]);
                        // hand the band's last scanline T_b to the next wavefront / workgroup
                        const int32_t il = s - (RPW - 1);
                        if (il >= 0 && il < W) {                 // wave-uniform
                            if constexpr (!OG) {
                                // ring space: the consumer's count only grows, so the last value
                                // read stays a valid lower bound; read LDS only when it is short
                                if (taken < il + 1 - R) {
                                    uint32_t spins = 0;
#pragma nounroll
                                    while ((taken = lds_get(cons + wave + 1)) < il + 1 - R) {
                                        if (++spins > SPIN_LIMIT) {
                                            raise_error(a.error);
                                            break;
                                        }
                                    }
                                }
                                int32_t* dst = hands ? ring_out + (size_t)(il & (R - 1)) * QT : trash + l;
#pragma unroll
                                for (int ky = 0; ky < KY; ++ky)
#pragma unroll
                                    for (int kx = 0; kx < KX; ++kx) dst[(ky * KX + kx) * G] = out[ky][kx];
                                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                                lds_put(prod + wave, il + 1);
                            } else {
                                if (gout && (((il + 1) & (a.chunk - 1)) == 0 || il == W - 1)) {
                                    // the row went out with device-scope stores: once they have
                                    // completed the progress word may show it
                                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                                    __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
                                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                                    if (lane == 0)
                                        flag_put(progress + super, epoch + (uint32_t)(il + 1));
                                }
                            }
                        }
                        if constexpr (!IG) {
                            if (s + 1 < W) read_input(s + 1);
                        }
                        fetch(s + PF, rc[u], rma[u], rmb[u], rb[u], rsh[u]);
                    }
                }
            };
            if (in_global) {
                if (out_lds) run(std::true_type{}, std::false_type{});
                else run(std::true_type{}, std::true_type{});
            } else {
                if (out_lds) run(std::false_type{}, std::false_type{});
                else run(std::false_type{}, std::true_type{});
            }
        }

        // Band complete: every wavefront makes its stores visible to the device before the
        // workgroup records the scan as done for this band (read by a fused second scan).
        if (a.npass > 1 && !second) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (a.npass > 1 && !second && threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            flag_put(done + super, (uint32_t)pass_index + 1);
        }
    }
}

// Marginal of eq. DP_2D_1 and its smallest argmin.  WIN: frames of the label-window
// solve; only the win x win window counts, and the label is read through the centre.
template <class T, class CT, bool WIN = false>
__global__ __launch_bounds__(256) void edp_aggregate_kernel(const AggArgs a) {
    constexpr int G = T::G, KX = T::KX, KY = T::KY, QT = T::QT;
    constexpr int RPW = 64 / G;
    const int32_t lane = lane_id();
    const int32_t grp = lane / G, l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t blk = (int32_t)blockIdx.x;
    const InstDesc d = a.ndesc > 0 ? uniform_desc(a.descs[find_instance(a.descs, a.ndesc, blk, 1)]) : a.one;
    const int32_t W = d.W, H = d.H, Q = d.qx * d.qy;
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t cells = W * H;
    const int32_t cell = (blk - d.first_block) * a.cells_per_block + wave * RPW + grp;
    const bool ok = cell < cells;
    const int32_t y = ok ? cell / W : 0, x = ok ? cell % W : 0;
    int32_t ox = 0, oy = 0;                        // window origin in the full label space
    if constexpr (WIN) {
        if (ok) {
            ox = d.centers[2 * cell] - d.win / 2;
            oy = d.centers[2 * cell + 1] - d.win / 2;
        }
    }
    // one vector load per operand: the lane's E sums of each neighbour are contiguous (lane-major),
    // its costs are KX-runs; a missing neighbour reads as 0 (out-of-range buffer offset)
    const int32_t tbytes = W * H * QT * 4;
    const int32_t lofs = l * T::E * 4;
    int32_t acc[KY][KX], tv[KY][KX];
#pragma unroll
    for (int ky = 0; ky < KY; ++ky) {
        const int32_t vy = py * KY + ky;
        const int32_t crun = (ok && vy < d.qy && px * KX < d.qx) ? (cell * Q + vy * d.qx + px * KX) * (int32_t)sizeof(CT)
                                                                 : OOB;
        int32_t cw[KX];
        load_cost_words<CT, KX>(make_rsrc(d.cost, cells * Q * (int32_t)sizeof(CT)), crun, cw);
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) acc[ky][kx] = cw[kx];
    }
    const int32_t nb[4] = {ok && x > 0 ? cell - 1 : -1, ok && x + 1 < W ? cell + 1 : -1,
                           ok && y > 0 ? cell - W : -1, ok && y + 1 < H ? cell + W : -1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        load_vec<T::E>(make_rsrc(d.t[k], tbytes), nb[k] >= 0 ? nb[k] * QT * 4 + lofs : OOB, &tv[0][0]);
#pragma unroll
        for (int ky = 0; ky < KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) acc[ky][kx] += tv[ky][kx];
    }
    int32_t best = 0x7FFFFFFF, bq = 0x7FFFFFFF;
#pragma unroll
    for (int ky = 0; ky < KY; ++ky)
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) {
            const int32_t vy = py * KY + ky, vx = px * KX + kx;
            const bool in = WIN ? (vx < d.win && vy < d.win) : (vx < d.qx && vy < d.qy);
            const int32_t lab = WIN ? (oy + vy) * d.qx_full + (ox + vx) : vy * d.qx + vx;
            const int32_t v = acc[ky][kx];
            if (ok && in && (v < best || (v == best && lab < bq))) {
                best = v;
                bq = lab;
            }
        }
    // smallest value, then the smallest label among the lanes holding it
    const int32_t vmin = group_min<T>(best, lane);
    const int32_t qmin = group_min<T>(best == vmin ? bq : 0x7FFFFFFF, lane);
    if (ok && l == 0) d.labels[cell] = qmin;
}

// Prefetch depth: enough steps in flight to cover the memory latency, within
// the 63 outstanding vector memory operations a wavefront can count.
template <class T>
constexpr int pass_pf() { return T::E <= 4 ? 8 : (T::E <= 8 ? 4 : 2); }

size_t pass_lds_bytes(int qt, int waves, int ring) {
    return (size_t)(2 * MAX_WAVES + 4 + qt) * 4 + (size_t)(waves > 1 ? waves - 1 : 0) * ring * qt * 4;
}
// the window solve adds a shifted-read area of 2 x 64 x 2 ints per wavefront
static size_t win_lds_bytes(int waves) { return (size_t)waves * 2 * 64 * 2 * 4; }

template <class T, class CK, int SPLIT>
static hipError_t run_pass(const PassArgs& a, int grid, int waves, hipStream_t s) {
    const size_t lds = pass_lds_bytes(T::QT, waves, a.ring);
    hipLaunchKernelGGL((edp_pass_kernel<T, CK, SPLIT, pass_pf<T>()>), dim3(grid), dim3(64 * waves), lds, s, a);
    return hipGetLastError();
}

using WinTile = Tile<4, 2, 4, 2>;

static hipError_t run_pass_win(const PassArgs& a, int grid, int waves, hipStream_t s) {
    const size_t lds = pass_lds_bytes(WinTile::QT, waves, a.ring) + win_lds_bytes(waves);
    hipLaunchKernelGGL((edp_pass_kernel<WinTile, int32_t, 1, pass_pf<WinTile>(), true>), dim3(grid), dim3(64 * waves),
                       lds, s, a);
    return hipGetLastError();
}

template <class T, class CT>
static hipError_t run_agg(const AggArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((edp_aggregate_kernel<T, CT>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class T, class CK, int SPLIT>
static int pass_occupancy(int waves, size_t lds) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, edp_pass_kernel<T, CK, SPLIT, pass_pf<T>()>,
                                                     64 * waves, lds) != hipSuccess)
        blocks = 1;
    return blocks < 1 ? 1 : blocks;
}

// SPLIT = 2 needs both halves of a vertex in one wavefront.
template <class T, class CK>
static hipError_t dispatch_pass(int split, const PassArgs& a, int grid, int waves, hipStream_t s) {
    if (split == 2) {
        if constexpr (2 * T::G <= 64) return run_pass<T, CK, 2>(a, grid, waves, s);
        return hipErrorInvalidValue;
    }
    return run_pass<T, CK, 1>(a, grid, waves, s);
}

template <class T, class CK>
static int dispatch_occupancy(int split, int waves, size_t lds) {
    if (split == 2) {
        if constexpr (2 * T::G <= 64) return pass_occupancy<T, CK, 2>(waves, lds);
        return 1;
    }
    return pass_occupancy<T, CK, 1>(waves, lds);
}

// cost kind: 1 int16 (element loads), 2 int32, 3 int16 in aligned pairs
template <class T>
static hipError_t dispatch_kind(int kind, int split, const PassArgs& a, int grid, int waves, hipStream_t s) {
    if (kind == 1) return dispatch_pass<T, int16_t>(split, a, grid, waves, s);
    if (kind == 3) {
        if constexpr (T::KX % 2 == 0) return dispatch_pass<T, Pair16>(split, a, grid, waves, s);
        return hipErrorInvalidValue;
    }
    return dispatch_pass<T, int32_t>(split, a, grid, waves, s);
}
template <class T>
static int occupancy_kind(int kind, int split, int waves, size_t lds) {
    if (kind == 1) return dispatch_occupancy<T, int16_t>(split, waves, lds);
    if (kind == 3) {
        if constexpr (T::KX % 2 == 0) return dispatch_occupancy<T, Pair16>(split, waves, lds);
        return 1;
    }
    return dispatch_occupancy<T, int32_t>(split, waves, lds);
}

hipError_t launch_edp_pass(int tile, int dtype, int split, const PassArgs& a, int grid, int waves,
                           hipStream_t s) {
    if (waves < 1 || waves > MAX_WAVES) return hipErrorInvalidValue;
    if (dtype == KIND_WINDOW) return tile == WIN_TILE && split == 1 ? run_pass_win(a, grid, waves, s) : hipErrorInvalidValue;
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky) \
    case id:                         \
        return dispatch_kind<Tile<px, kx, py, ky>>(dtype, split, a, grid, waves, s);
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_edp_aggregate_win(const AggArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((edp_aggregate_kernel<WinTile, int32_t, true>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
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

int pass_capacity(int tile, int dtype, int split, int waves, size_t lds_bytes) {
    int per_cu = 1;
    if (dtype == KIND_WINDOW) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, edp_pass_kernel<WinTile, int32_t, 1, pass_pf<WinTile>(), true>, 64 * waves,
                lds_bytes + win_lds_bytes(waves)) != hipSuccess || per_cu < 1)
            per_cu = 1;
        tile = -1;
    }
    switch (tile) {
#define EDP_CASE(id, px, kx, py, ky)                                               \
    case id:                                                                       \
        per_cu = occupancy_kind<Tile<px, kx, py, ky>>(dtype, split, waves, lds_bytes); \
        break;
        EDP_TILE_LIST(EDP_CASE)
#undef EDP_CASE
    }
    int dev = 0, cus = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1;
    return per_cu * cus;
}

}  // namespace edp
