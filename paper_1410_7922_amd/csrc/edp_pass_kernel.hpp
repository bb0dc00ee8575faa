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
//  * Workgroup: its compute wavefronts take consecutive bands of scanlines;
//    the last scanline of a band hands T_b to the next wavefront through an
//    LDS ring (counters in LDS).  Workgroups take whole groups of bands in
//    scan order from a ticket counter, so the group a workgroup waits on is
//    always held by a running workgroup.  Two more wavefronts per workgroup
//    move rows between workgroups: one stores the last band's T_b with
//    device-scope stores and publishes the column count once they have
//    completed, the other reads the row above the first band with
//    device-scope loads into the first ring as the workgroup above publishes
//    it.  The compute wavefronts thus only wait on LDS counters and on their
//    own prefetched loads.
// T_b written by P1 and P3 is only read inside the scan, so it reaches memory
// only at workgroup boundaries.  Operands that do not depend on the scan (C
// and the two "old" arrays) are prefetched PF steps ahead in a register ring.
#pragma once
#include "edp_device.hpp"
#include "edp_internal.hpp"

namespace edp {

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
// Tagged sums handed between workgroups: (value, tag) in one 64-bit word, stored and loaded as
// single device-scope 64-bit accesses, so a reader that sees the tag sees the value stored with it.
typedef __attribute__((address_space(1))) unsigned long long gu64;
__device__ __forceinline__ unsigned long long tag_get(const unsigned long long* p) {
    return __hip_atomic_load((const gu64*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void tag_put(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store((gu64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// WIN: the label-window solve.  Every vertex holds an 8 x 8 frame of labels around its own
// window (costs outside the window are large), d.aux holds the frame shifts towards the four
// neighbours, and each sum handed on is evaluated in the receiving vertex's frame.
//
// A workgroup has NW compute wavefronts and two helper wavefronts (the last two).  Compute
// wavefront k reads the T_b row above its band from LDS ring k and writes its band's last
// scanline into ring k + 1.  The row-in helper fills ring 0 from memory as the workgroup
// band above publishes its progress (zeros above the first band); the row-out helper
// empties the ring of the last active wavefront into memory and publishes progress once its
// stores have completed.  The compute wavefronts never touch another workgroup's data, so
// they never wait for memory operations other than their own prefetched loads.
template <class T, class CK, int SPLIT, int PF, bool WIN = false, int MS = MS_LINEAR>
__global__ __launch_bounds__(64 * (MAX_WAVES + 2)) void edp_pass_kernel(const PassArgs a) {
    constexpr int G = T::G, KX = T::KX, KR = T::KR, E = T::E, QT = T::QT;
    constexpr int CL = SPLIT * G;                  // lanes per vertex
    constexpr int RPW = 64 / CL;                   // scanlines per wavefront
    constexpr int CB = CostBytes<CK>::value;
    static_assert(CL <= 64, "vertex wider than a wavefront");
    extern __shared__ int32_t lds[];
    int32_t* wr = lds;                             // [MAX_WAVES + 1] columns written into ring k
    int32_t* rd = lds + (MAX_WAVES + 1);           // [MAX_WAVES + 1] columns taken from ring k
    int32_t* misc = lds + 2 * (MAX_WAVES + 1);     // [0] ticket broadcast
    int32_t* trash = misc + 4;                     // [QT] sink of the lanes that hand nothing over
    int32_t* rings = trash + QT;                   // [NW + 1][ring][QT]
    static_assert(!WIN || SPLIT == 1, "the window solve runs both searches on every lane");

    const int32_t lane = lane_id();
    // wavefront-uniform values live in scalar registers, so control flow on them is scalar
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t NW = (int32_t)(blockDim.x >> 6) - 2;     // compute wavefronts; waves NW, NW + 1 help
    const int32_t grp = lane / CL;
    const bool beta = SPLIT == 2 && ((lane / G) & 1);
    const int32_t l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t R = a.ring;
    // T arrays are lane-major inside a vertex: the lane's E labels are contiguous
    const int32_t lofs = l * E * 4;

    for (;;) {
        if (threadIdx.x == 0) misc[0] = (int32_t)atomicAdd(a.ticket, 1u);
        if (threadIdx.x < 2 * (MAX_WAVES + 1)) lds[threadIdx.x] = 0;
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
        const int32_t W = d.W, H = d.H, Q = d.qx * d.qy * d.qz;
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
        // Buffer resources: a lane whose operand does not exist uses offset OOB, so
        // its load returns 0 and its store is dropped, with no branch around it.
        const int32_t tbytes = W * H * QT * 4;         // below 2^31 (checked by the host)
        // ka is 0 or 1 and kb 2 or 3: pick the arrays with selects (no indexed private array)
        int32_t* const t_b = kb == 3 ? d.t[3] : d.t[2];
        const __amdgpu_buffer_rsrc_t rs_b = make_rsrc(t_b, tbytes);
        const int32_t nact = min(NW, d.nbands - super * NW);   // compute wavefronts with a band
        if (wave >= NW) {
            // Helpers (wave NW: rows in, wave NW + 1: rows out).  Lanes move CPI columns per
            // instruction, G lanes x E values each; a ring slot holds value (ky, kx) of vertex
            // lane l at (ky * KX + kx) * G + l.
            constexpr int CPI = 64 / G;
            constexpr int NI = CPI >= 4 ? 2 : 8 / CPI; // instructions per batch
            const int32_t cg = lane / G;
            const int32_t xs = sx > 0 ? 0 : W - 1;     // x of column 0
            const int32_t dtc = sx * QT * 4;           // byte stride per column
            uint32_t idle = 0;
            if (wave == NW) {
                const bool gin = super > 0;            // a workgroup band above exists
                const int32_t j0 = super * NW * RPW;   // first scanline of the band
                const int32_t b_in = gin ? cell_off(((sy > 0 ? j0 : H - 1 - j0) - sy) * W + xs, QT * 4) + lofs : OOB;
                int32_t* const ring0 = rings + l;
                int32_t cin = 0;
                uint32_t seen = 0;
                if (!gin) {
                    // nothing above the first band: ring 0 holds zeros, all columns at once
                    for (int32_t k = lane; k < R * QT; k += 64) rings[k] = 0;
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    lds_put(wr, W);
                    cin = W;
                }
                // tagged rows (d.hand): column c of the row above carries tag epoch + c + 1 in every
                // word; the buffer is cleared before each solve, so no other tag can match
                const unsigned long long* const hin =
                    d.hand && gin ? d.hand + (size_t)(((second ? 1 : 0) * (d.nsuper - 1) + super - 1) * W) * QT + l * E
                                  : nullptr;
                // at most 32 tagged words per lane in flight (the scan's register budget)
                constexpr int NIT = NI * E <= 32 ? NI : (E >= 32 ? 1 : 32 / E);
#pragma nounroll
                while (hin && cin < W) {
                    const int32_t n = min(min(W - cin, lds_get(rd) + R - cin), NIT * CPI);
                    int32_t got = 0;
                    if (n > 0) {
                        int32_t v[NIT][E];
                        unsigned long long okm[NIT];
#pragma unroll
                        for (int q = 0; q < NIT; ++q) {
                            const int32_t c = q * CPI + cg;
                            bool good = c < n;
                            const uint32_t tag = epoch + (uint32_t)(cin + c) + 1u;
#pragma unroll
                            for (int k = 0; k < E; ++k) {
                                const unsigned long long x = c < n ? tag_get(hin + (size_t)(cin + c) * QT + k) : 0ull;
                                v[q][k] = (int32_t)(uint32_t)x;
                                good = good && (uint32_t)(x >> 32) == tag;
                            }
                            okm[q] = __ballot(good);
                        }
                        // columns arrive in any order: take the leading run whose every lane is tagged
                        constexpr unsigned long long GM = G == 64 ? ~0ull : (1ull << G) - 1;
                        bool run = true;
#pragma unroll
                        for (int q = 0; q < NIT; ++q)
#pragma unroll
                            for (int g = 0; g < CPI; ++g) {
                                run = run && q * CPI + g < n && ((okm[q] >> (g * G)) & GM) == GM;
                                if (run) got = q * CPI + g + 1;
                            }
#pragma unroll
                        for (int q = 0; q < NIT; ++q) {
                            const int32_t c = q * CPI + cg;
                            if (c < got) {
                                int32_t* slot = ring0 + (size_t)((cin + c) & (R - 1)) * QT;
#pragma unroll
                                for (int k = 0; k < E; ++k) slot[k * G] = v[q][k];
                            }
                        }
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        if (got > 0) lds_put(wr, cin + got);
                        cin += got;
                    }
                    if (got > 0) {
                        idle = 0;
                    } else {
                        if (++idle > SPIN_LIMIT_BAND || ((idle & 1023) == 0 && flag_get(a.error) != 0)) {
                            raise_error(a.error);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
#pragma nounroll
                while (!hin && cin < W) {
                    if (seen <= (uint32_t)cin) {
                        const uint32_t v = __builtin_amdgcn_readfirstlane(flag_get(progress + super - 1));
                        seen = v > epoch ? v - epoch : 0u;
                    }
                    int32_t n = min((int32_t)seen - cin, lds_get(rd) + R - cin);
                    n = min(n, NI * CPI);
                    if (n > 0) {
                        // the row is read with device-scope loads issued after the progress word
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        int32_t v[NI][E];
#pragma unroll
                        for (int q = 0; q < NI; ++q) {
                            const int32_t c = q * CPI + cg;
                            load_vec<E, CPOL_DEVICE>(rs_b, c < n ? b_in + (cin + c) * dtc : OOB, v[q]);
                        }
#pragma unroll
                        for (int q = 0; q < NI; ++q) {
                            const int32_t c = q * CPI + cg;
                            if (c < n) {
                                int32_t* slot = ring0 + (size_t)((cin + c) & (R - 1)) * QT;
#pragma unroll
                                for (int k = 0; k < E; ++k) slot[k * G] = v[q][k];
                            }
                        }
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        lds_put(wr, cin + n);
                        cin += n;
                        idle = 0;
                    } else {
                        // give up (and let every other waiter give up) instead of hanging
                        if (++idle > SPIN_LIMIT_BAND || ((idle & 1023) == 0 && flag_get(a.error) != 0)) {
                            raise_error(a.error);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            } else {
                const bool gout = super * NW + nact < d.nbands;   // a workgroup band below exists
                const int32_t j1 = (super * NW + nact) * RPW - 1;   // last scanline (full band if gout)
                const int32_t b_out = gout ? cell_off((sy > 0 ? j1 : H - 1 - j1) * W + xs, QT * 4) + lofs : OOB;
                const int32_t* const ring_last = rings + (size_t)nact * R * QT + l;
                unsigned long long* const hout =
                    d.hand && gout ? d.hand + (size_t)(((second ? 1 : 0) * (d.nsuper - 1) + super) * W) * QT + l * E
                                   : nullptr;
                int32_t cout = 0, pub = 0;
#pragma nounroll
                while (cout < W) {
                    const int32_t n = min(lds_get(wr + nact) - cout, NI * CPI);
                    if (n > 0) {
#pragma unroll
                        for (int q = 0; q < NI; ++q) {
                            const int32_t c = q * CPI + cg;
                            const int32_t* slot = ring_last + (size_t)((cout + c) & (R - 1)) * QT;
                            int32_t v[E];
#pragma unroll
                            for (int k = 0; k < E; ++k) v[k] = slot[k * G];
                            if (hout) {
                                if (c < n) {
                                    const unsigned long long tag = (unsigned long long)(epoch + (uint32_t)(cout + c) + 1u) << 32;
#pragma unroll
                                    for (int k = 0; k < E; ++k)
                                        tag_put(hout + (size_t)(cout + c) * QT + k, tag | (uint32_t)v[k]);
                                }
                            } else {
                                store_vec<E, CPOL_DEVICE>(rs_b, c < n ? b_out + (cout + c) * dtc : OOB, v);
                            }
                        }
                        // LDS operations of a wavefront complete in order: the slots are read
                        // before the count that frees them is written
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        lds_put(rd + nact, cout + n);
                        cout += n;
                        if (!hout && gout && (cout - pub >= a.chunk || cout == W)) {
                            // the row went out with device-scope stores: once they have
                            // completed the progress word may show it
                            __atomic_signal_fence(__ATOMIC_SEQ_CST);
                            __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
                            __atomic_signal_fence(__ATOMIC_SEQ_CST);
                            if (lane == 0) flag_put(progress + super, epoch + (uint32_t)cout);
                            pub = cout;
                        }
                        idle = 0;
                    } else {
                        if (++idle > SPIN_LIMIT_BAND || ((idle & 1023) == 0 && flag_get(a.error) != 0)) {
                            raise_error(a.error);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            }
        } else if (wave < nact) {
            const int32_t band = super * NW + wave;
            const bool joint = d.joint != 0;
            const LineIndex<T> li(d.lam, lane);
            const WinPen sp(d.lam, d.trunc, d.qx, d.qy, d.squared != 0, d.qz);   // general RMS window
            const __amdgpu_buffer_rsrc_t rs_c = make_rsrc(d.cost, W * H * Q * CB);
            int32_t* const t_a = ka ? d.t[1] : d.t[0];
            int32_t* const t_ma = ka ? d.t[0] : d.t[1];
            int32_t* const t_mb = kb == 3 ? d.t[2] : d.t[3];
            // an operand that is zero (no earlier scan) or a sum that nobody reads later gets an
            // empty buffer: its loads return 0 and its stores are dropped, with no per-step test
            const __amdgpu_buffer_rsrc_t rs_a = make_rsrc(t_a, tbytes);
            const __amdgpu_buffer_rsrc_t rs_ma = make_rsrc(t_ma, old_a_zero ? 0 : tbytes);
            const __amdgpu_buffer_rsrc_t rs_mb = make_rsrc(t_mb, old_b_zero ? 0 : tbytes);
            const __amdgpu_buffer_rsrc_t rs_bo = make_rsrc(t_b, b_live ? tbytes : 0);
            int32_t crun[KR];                              // cost byte offset of the lane's run of KX labels
            bool valid[KR][KX];
#pragma unroll
            for (int r = 0; r < KR; ++r) {                 // row r: vz = r / KY, vy = py KY + r % KY
                const int32_t vy = py * T::KY + r % T::KY, vz = r / T::KY;
                const bool rin = vy < d.qy && vz < d.qz;
                crun[r] = (rin && px * KX < d.qx) ? ((vz * d.qy + vy) * d.qx + px * KX) * CB : OOB;
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) valid[r][kx] = px * KX + kx < d.qx && rin;
            }
            const int32_t j = band * RPW + grp;            // scan-order row index
            // a lane whose labels are all padding neither loads nor stores sums: its values are
            // replaced by PADV before every use
            const bool rowok = j < H && px * KX < d.qx && py * T::KY < d.qy;
            const int32_t y = sy > 0 ? j : H - 1 - j;
            const int32_t yn = y + sy;                     // next row in scan order
            const bool has_next = j + 1 < H;
            const bool store_a = SPLIT == 1 || !beta;
            const bool store_b = SPLIT == 1 || beta;
            // the lanes of the band's last scanline that carry T_b hand it on
            const bool hands = grp == RPW - 1 && (SPLIT == 1 || beta);
            const int32_t* ring_in = rings + (size_t)wave * R * QT + l;
            int32_t* ring_out = rings + (size_t)(wave + 1) * R * QT + l;
            // byte offsets at step 0 (column -grp) and per-step strides: at step t the lane's
            // vertex is x = x0 + sx (t - grp) of row y
            const int32_t x0 = (sx > 0 ? 0 : W - 1) - sx * grp;
            const int32_t dc = sx * Q * CB, dt = sx * QT * 4;
            const int32_t bc = cell_off(y * W + x0, Q * CB);
            const int32_t bt = cell_off(y * W + x0, QT * 4) + lofs;
            const int32_t ba = bt + dt;                    // (x + sx, y)
            const int32_t bb = cell_off(yn * W + x0, QT * 4) + lofs;
            // window solve: frame-shift codes of the vertex (8 bytes per vertex)
            const int32_t bsh = cell_off(y * W + x0, 8), dsh = sx * 8;
            const __amdgpu_buffer_rsrc_t rs_sh = make_rsrc(d.aux, WIN ? W * H * 8 : 0);
            int32_t* const wscr = rings + (size_t)(NW + 1) * R * QT + (size_t)wave * 2 * 64 * (KX > KR ? KX : KR);
            // steps rounded up to whole prefetch rounds: the extra steps touch nothing (every lane
            // is past the end of its row), and a fixed count of loads per step lets the compiler
            // wait for exactly the slot in use instead of for every load in flight
            const int32_t nsteps = (W + RPW - 1 + PF - 1) / PF * PF;
            int32_t taken = 0;                             // columns the next wavefront has taken (lower bound)

            constexpr int CW = CostWords<CK, KX>::value;
            int32_t rc[PF][KR][CW], rma[PF][KR][KX], rmb[PF][KR][KX];
            int32_t rsh[PF][WIN ? 2 : 1];
            int32_t carry[KR][KX], out[KR][KX];
#pragma unroll
            for (int ky = 0; ky < KR; ++ky)
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) carry[ky][kx] = out[ky][kx] = 0;

            // Issue the loads of step t into one ring slot (no branch around a load).
            // STEADY: every scanline of the wavefront is strictly inside its row at column t
            // (0 < t - grp < W - 1), which the caller knows for a whole round of steps
            auto fetch = [&](auto steady, const int32_t t, int32_t (&c)[KR][CW], int32_t (&ma)[KR][KX],
                             int32_t (&mb)[KR][KX], int32_t (&sh)[WIN ? 2 : 1]) {
                constexpr bool STEADY = decltype(steady)::value;
                // column i = t - grp of this lane's scanline; offsets move by a fixed stride per step
                const uint32_t i = (uint32_t)(t - grp);
                const bool act = STEADY ? rowok : rowok && i < (uint32_t)W;
                const bool nxt = STEADY || i + 1 < (uint32_t)W;     // the next column in scan order exists
                const int32_t offc = act ? bc + t * dc : OOB;
                const int32_t offa = (act && nxt) ? ba + t * dt : OOB;
                const int32_t offb = (act && has_next) ? bb + t * dt : OOB;
#pragma unroll
                for (int ky = 0; ky < KR; ++ky) load_cost_words<CK, KX>(rs_c, offc + crun[ky], c[ky]);
                load_vec<E>(rs_ma, offa, &ma[0][0]);
                load_vec<E>(rs_mb, offb, &mb[0][0]);
                if constexpr (WIN) load_vec<2>(rs_sh, act ? bsh + t * dsh : OOB, sh);
            };
#pragma unroll
            for (int u = 0; u < PF; ++u) fetch(std::false_type{}, u, rc[u], rma[u], rmb[u], rsh[u]);

            // Input: the producer's count and the ring slot of column t, read back to back.  LDS
            // performs the operations of the CU in arrival order and the producer writes a slot
            // before its count, so when the count shows column t the slot read issued after it
            // returns that column.  Column t + 1 is read at the end of step t, which keeps the
            // LDS round trip off the step when the producer is ahead.
            int32_t in_ready = 0, in_lb[KR][KX];
            auto read_input = [&](const int32_t t) {
                const int32_t* slot = ring_in + (size_t)(t & (R - 1)) * QT;
                in_ready = lds_get(wr + wave);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
                for (int ky = 0; ky < KR; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx)
                        in_lb[ky][kx] = slot[(ky * KX + kx) * G];
            };
            read_input(0);

            auto step = [&](auto steady, const int u, const int32_t s) {
                constexpr bool STEADY = decltype(steady)::value;
                const int32_t i = s - grp;
                const bool act = STEADY ? rowok : rowok && (uint32_t)i < (uint32_t)W;
                // T_b of the row above at this column, for group 0
                int32_t lb[KR][KX];
#pragma unroll
                for (int ky = 0; ky < KR; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) lb[ky][kx] = 0;
                if (STEADY || s < W) {                       // wave-uniform
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
                    for (int ky = 0; ky < KR; ++ky)
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx) lb[ky][kx] = in_lb[ky][kx];
                    // LDS operations of a wavefront complete in order: the slot is read
                    // before the count that frees it is written
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    lds_put(rd + wave, s + 1);
                }
                int32_t h[KR][KX], h2[KR][KX];
#pragma unroll
                for (int ky = 0; ky < KR; ++ky)
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
                            if (!STEADY && i == 0) cr = 0;
                        }
                        if (grp == 0) mb = lb[ky][kx];
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
                    if constexpr (MS == MS_WINDOW) {
                        min_search_shift_window<T>(h, sp, d.clipd, joint, lane, dxa, dya);
                        min_search_shift_window<T>(h2, sp, d.clipd, joint, lane, dxb, dyb);
                    } else {
                        min_search_shift<T>(h, d.lam, d.clipd, joint, lane, dxa, dya, wscr);
                        min_search_shift<T>(h2, d.lam, d.clipd, joint, lane, dxb, dyb, wscr);
                    }
                } else if constexpr (MS != MS_LINEAR) {
                    constexpr int NWK = MS == MS_WALK ? 0 : (MS == MS_WINDOW1 ? 1 : 2);
                    min_search_window<T, NWK>(h, sp, d.clipd, joint, lane);
                    if constexpr (SPLIT == 1) min_search_window<T, NWK>(h2, sp, d.clipd, joint, lane);
                } else {
                    min_search<T>(h, li, d.clipd, joint, lane);
                    if constexpr (SPLIT == 1) min_search<T>(h2, li, d.clipd, joint, lane);
                }
                const int32_t o = bt + s * dt;
                const int32_t oa = (act && store_a) ? o : OOB;
                const int32_t ob = (act && store_b) ? o : OOB;
                int32_t tbv[KR][KX];
#pragma unroll
                for (int ky = 0; ky < KR; ++ky)
#pragma unroll
                    for (int kx = 0; kx < KX; ++kx) {
                        tbv[ky][kx] = SPLIT == 1 ? h2[ky][kx] : h[ky][kx];
                        if constexpr (SPLIT == 1) carry[ky][kx] = act ? h[ky][kx] : carry[ky][kx];
                        out[ky][kx] = tbv[ky][kx];
                    }
                store_vec<E>(rs_a, oa, &h[0][0]);
                store_vec<E>(rs_bo, ob, &tbv[0][0]);
                // hand the band's last scanline T_b to the next wavefront (or the helper)
                const int32_t il = s - (RPW - 1);
                if (STEADY || (il >= 0 && il < W)) {         // wave-uniform
                    // ring space: the consumer's count only grows, so the last value read
                    // stays a valid lower bound; read LDS only when it is short
                    if (taken < il + 1 - R) {
                        uint32_t spins = 0;
#pragma nounroll
                        while ((taken = lds_get(rd + wave + 1)) < il + 1 - R) {
                            if (++spins > SPIN_LIMIT) {
                                raise_error(a.error);
                                break;
                            }
                        }
                    }
                    int32_t* dst = hands ? ring_out + (size_t)(il & (R - 1)) * QT : trash + l;
#pragma unroll
                    for (int ky = 0; ky < KR; ++ky)
#pragma unroll
                        for (int kx = 0; kx < KX; ++kx) dst[(ky * KX + kx) * G] = out[ky][kx];
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    lds_put(wr + wave + 1, il + 1);
                }
                if (STEADY || s + 1 < W) read_input(s + 1);
                fetch(steady, s + PF, rc[u], rma[u], rmb[u], rsh[u]);
            };
            // a steady round: its steps and the steps it prefetches for have every scanline of the
            // wavefront strictly inside its row (s0 >= RPW, s0 + 2 PF + 1 <= W).  Only tiles with
            // few labels per lane get the second copy of the round (the others would spill).
            constexpr bool TWO_COPIES = E <= 2 || (E <= 4 && G <= 16);
            auto is_steady = [&](int32_t s0) { return s0 >= RPW && s0 + 2 * PF + 1 <= W; };
            if constexpr (TWO_COPIES && !WIN) {
                // the steady rounds are one run of consecutive rounds: the rounds before it, the
                // run and the rounds after it are three loops, each with a single copy of the
                // round, so the prefetch registers of a round are those of the next (one loop with
                // both copies moved them between rounds, after waiting for every load in flight)
                int32_t s0 = 0;
                for (; s0 < nsteps && !is_steady(s0); s0 += PF) {
#pragma unroll
                    for (int u = 0; u < PF; ++u) step(std::false_type{}, u, s0 + u);
                }
                for (; s0 < nsteps && is_steady(s0); s0 += PF) {
#pragma unroll
                    for (int u = 0; u < PF; ++u) step(std::true_type{}, u, s0 + u);
                }
                for (; s0 < nsteps; s0 += PF) {
#pragma unroll
                    for (int u = 0; u < PF; ++u) step(std::false_type{}, u, s0 + u);
                }
            } else {
                // one loop: tiles without the steady copy, and the window solve (which ran
                // slower as three loops)
                for (int32_t s0 = 0; s0 < nsteps; s0 += PF) {
                    if (TWO_COPIES && is_steady(s0)) {
                        if constexpr (TWO_COPIES) {
#pragma unroll
                            for (int u = 0; u < PF; ++u) step(std::true_type{}, u, s0 + u);
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < PF; ++u) step(std::false_type{}, u, s0 + u);
                    }
                }
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
    constexpr int G = T::G, KX = T::KX, KR = T::KR, QT = T::QT;
    constexpr int RPW = 64 / G;
    const int32_t lane = lane_id();
    const int32_t grp = lane / G, l = lane % G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t blk = (int32_t)blockIdx.x;
    const InstDesc d = a.ndesc > 0 ? uniform_desc(a.descs[find_instance(a.descs, a.ndesc, blk, 1)]) : a.one;
    const int32_t W = d.W, H = d.H, Q = d.qx * d.qy * d.qz;
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t cells = W * H;
    // the scans ran before this launch on the same stream: their error word is final
    if (threadIdx.x == 0 && blk == d.first_block && d.status)
        *d.status = (a.error && *a.error != 0) ? STATUS_TIMEOUT : 0;
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
    int32_t acc[KR][KX], tv[KR][KX];
#pragma unroll
    for (int r = 0; r < KR; ++r) {                 // row r: vz = r / KY, vy = py KY + r % KY
        const int32_t vy = py * T::KY + r % T::KY, vz = r / T::KY;
        const int32_t crun = (ok && vy < d.qy && vz < d.qz && px * KX < d.qx)
                                 ? (cell * Q + (vz * d.qy + vy) * d.qx + px * KX) * (int32_t)sizeof(CT)
                                 : OOB;
        int32_t cw[KX];
        load_cost_words<CT, KX>(make_rsrc(d.cost, cells * Q * (int32_t)sizeof(CT)), crun, cw);
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) acc[r][kx] = cw[kx];
    }
    // lanes whose labels are all padding (or, in a window solve, all outside the window) read
    // no sums: their values never reach the argmin
    const bool live = WIN ? (px * KX < d.win && py * T::KY < d.win) : (px * KX < d.qx && py * T::KY < d.qy);
    const bool rd = ok && live;
    const int32_t nb[4] = {rd && x > 0 ? cell - 1 : -1, rd && x + 1 < W ? cell + 1 : -1,
                           rd && y > 0 ? cell - W : -1, rd && y + 1 < H ? cell + W : -1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        load_vec<T::E>(make_rsrc(d.t[k], tbytes), nb[k] >= 0 ? nb[k] * QT * 4 + lofs : OOB, &tv[0][0]);
#pragma unroll
        for (int ky = 0; ky < KR; ++ky)
#pragma unroll
            for (int kx = 0; kx < KX; ++kx) acc[ky][kx] += tv[ky][kx];
    }
    int32_t best = 0x7FFFFFFF, bq = 0x7FFFFFFF;
#pragma unroll
    for (int r = 0; r < KR; ++r)
#pragma unroll
        for (int kx = 0; kx < KX; ++kx) {
            const int32_t vy = py * T::KY + r % T::KY, vz = r / T::KY, vx = px * KX + kx;
            const bool in = WIN ? (vx < d.win && vy < d.win) : (vx < d.qx && vy < d.qy && vz < d.qz);
            const int32_t lab = WIN ? (oy + vy) * d.qx_full + (ox + vx) : (vz * d.qy + vy) * d.qx + vx;
            const int32_t v = acc[r][kx];
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

// the window solve adds a shifted-read area of 2 x 64 x 2 ints per wavefront
inline size_t win_lds_bytes(int waves) { return (size_t)waves * 2 * 64 * 2 * 4; }

template <class T, class CK, int SPLIT, int MS>
static hipError_t run_pass(const PassArgs& a, int grid, int waves, hipStream_t s) {
    const size_t lds = pass_lds_bytes(T::QT, waves, a.ring);
    hipLaunchKernelGGL((edp_pass_kernel<T, CK, SPLIT, pass_pf<T>(), false, MS>), dim3(grid), dim3(64 * (waves + 2)),
                       lds, s, a);
    return hipGetLastError();
}



template <class T, class CT>
static hipError_t run_agg(const AggArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((edp_aggregate_kernel<T, CT>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class T, class CK, int SPLIT, int MS>
static int pass_occupancy(int waves, size_t lds) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, edp_pass_kernel<T, CK, SPLIT, pass_pf<T>(), false, MS>,
                                                     64 * (waves + 2), lds) != hipSuccess)
        blocks = 1;
    return blocks < 1 ? 1 : blocks;
}

// SPLIT = 2 needs both halves of a vertex in one wavefront.
template <class T, class CK, int MS>
static hipError_t dispatch_pass(int split, const PassArgs& a, int grid, int waves, hipStream_t s) {
    if (split == 2) {
        if constexpr (2 * T::G <= 64) return run_pass<T, CK, 2, MS>(a, grid, waves, s);
        return hipErrorInvalidValue;
    }
    return run_pass<T, CK, 1, MS>(a, grid, waves, s);
}

template <class T, class CK, int MS>
static int dispatch_occupancy(int split, int waves, size_t lds) {
    if (split == 2) {
        if constexpr (2 * T::G <= 64) return pass_occupancy<T, CK, 2, MS>(waves, lds);
        return 1;
    }
    return pass_occupancy<T, CK, 1, MS>(waves, lds);
}

// cost kind: 1 int16 (element loads), 2 int32, 3 int16 in aligned pairs
template <class T, int MS>
static hipError_t dispatch_kind(int kind, int split, const PassArgs& a, int grid, int waves, hipStream_t s) {
    if (kind == 1) return dispatch_pass<T, int16_t, MS>(split, a, grid, waves, s);
    if (kind == 3) {
        if constexpr (T::KX % 2 == 0) return dispatch_pass<T, Pair16, MS>(split, a, grid, waves, s);
        return hipErrorInvalidValue;
    }
    return dispatch_pass<T, int32_t, MS>(split, a, grid, waves, s);
}
template <class T, int MS>
static int occupancy_kind(int kind, int split, int waves, size_t lds) {
    if (kind == 1) return dispatch_occupancy<T, int16_t, MS>(split, waves, lds);
    if (kind == 3) {
        if constexpr (T::KX % 2 == 0) return dispatch_occupancy<T, Pair16, MS>(split, waves, lds);
        return 1;
    }
    return dispatch_occupancy<T, int32_t, MS>(split, waves, lds);
}

// Per-tile entry points.  Each is instantiated explicitly in one of the edp_pass_t*.hip
// translation units (the kernels of a tile are large; the units compile in parallel).
template <int ID> struct TileOf;
#define EDP_TILE_OF(id, px, kx, py, ky) \
    template <> struct TileOf<id> { using type = Tile<px, kx, py, ky>; };
EDP_TILE_LIST(EDP_TILE_OF)
#undef EDP_TILE_OF
#define EDP_TILE3_OF(id, px, kx, py, ky, kz) \
    template <> struct TileOf<id> { using type = Tile<px, kx, py, ky, kz>; };
EDP_TILE3_LIST(EDP_TILE3_OF)
#undef EDP_TILE3_OF

// MS: the minimum search (MS_LINEAR, MS_WINDOW, MS_WALK)
template <int ID, int MS>
hipError_t pass_tile(int kind, int split, const PassArgs& a, int grid, int waves, hipStream_t s) {
    return dispatch_kind<typename TileOf<ID>::type, MS>(kind, split, a, grid, waves, s);
}
template <int ID, int MS>
int occupancy_tile(int kind, int split, int waves, size_t lds) {
    return occupancy_kind<typename TileOf<ID>::type, MS>(kind, split, waves, lds);
}
template <int ID>
hipError_t aggregate_tile(int dtype, const AggArgs& a, int grid, hipStream_t s) {
    using T = typename TileOf<ID>::type;
    return dtype == 1 ? run_agg<T, int16_t>(a, grid, s) : run_agg<T, int32_t>(a, grid, s);
}

// the label-window solve's 8 x 8 frames
using WinTile = TileOf<WIN_TILE>::type;

#define EDP_INSTANTIATE_TILE(id)                                                                         \
    template hipError_t pass_tile<id, MS_LINEAR>(int, int, const PassArgs&, int, int, hipStream_t);       \
    template int occupancy_tile<id, MS_LINEAR>(int, int, int, size_t);                                   \
    template hipError_t aggregate_tile<id>(int, const AggArgs&, int, hipStream_t);
// the scan kernels of a tile with the general RMS
#define EDP_INSTANTIATE_TILE_WIN(id)                                                                      \
    template hipError_t pass_tile<id, MS_WINDOW>(int, int, const PassArgs&, int, int, hipStream_t);     \
    template int occupancy_tile<id, MS_WINDOW>(int, int, int, size_t);                                 \
    template hipError_t pass_tile<id, MS_WALK>(int, int, const PassArgs&, int, int, hipStream_t);      \
    template int occupancy_tile<id, MS_WALK>(int, int, int, size_t);                                   \
    template hipError_t pass_tile<id, MS_WINDOW1>(int, int, const PassArgs&, int, int, hipStream_t);   \
    template int occupancy_tile<id, MS_WINDOW1>(int, int, int, size_t);

}  // namespace edp
