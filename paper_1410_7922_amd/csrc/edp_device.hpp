// Device building blocks for gfx950: lane tiles, cross-lane exchange, the
// linear recursive minimum search (Mozerov, arXiv 1410.7922, Sec. 3.2) and the
// general one (Sec. 3.1).
//
// A "lane tile" maps the labels of one DSI vertex onto a group of G = PX*PY
// lanes of a 64-wide wavefront.  Lane (px, py) of a group holds the KY x KX
// block of labels vy = py*KY + ky, vx = px*KX + kx, so a line of the label
// space along x lies in consecutive lanes of one lane row and a line along y
// in lanes PX apart.  A three-dimensional label space repeats the block for
// vz = 0 .. KZ-1 in every lane: the lane's KR = KZ*KY rows of KX labels are
// row r = kz*KY + ky, and a line along z lies inside one lane.
//
// Cross-lane exchange uses DPP inside 16-lane rows (row_shr / row_shl /
// row_ror / mirrors / quad permutes, a few cycles each) and the gfx950
// v_permlane16_swap / v_permlane32_swap instructions to move data between
// rows, and ds_bpermute where a move crosses rows and the permlane route would
// take several instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace edp {

// Value held by labels outside the label space.  It stays above every real
// value, and adding the largest distance penalty to it cannot overflow int32.
constexpr int32_t PADV = 0x3FFFFFFF;

template <int PX_, int KX_, int PY_, int KY_, int KZ_ = 1>
struct Tile {
    static constexpr int PX = PX_, KX = KX_, PY = PY_, KY = KY_, KZ = KZ_;
    static constexpr int KR = KZ * KY;         // rows of KX labels per lane
    static constexpr int G = PX * PY;          // lanes per vertex
    static constexpr int E = KX * KR;          // labels per lane
    static constexpr int QT = G * E;           // padded labels per vertex
    static_assert(G >= 1 && G <= 64 && (64 % G) == 0, "group must divide the wavefront");
    static_assert((PX & (PX - 1)) == 0 && (PY & (PY - 1)) == 0, "power-of-two lane grid");
    static_assert(PY == 1 || PX * PY >= 16, "y lines must fill whole 16-lane rows");
};

__device__ __forceinline__ int32_t lane_id() { return (int32_t)__lane_id(); }
__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ __forceinline__ int32_t imin3(int32_t a, int32_t b, int32_t c) { return imin(imin(a, b), c); }

// Raw buffer access.  Offsets are bytes; OOB lies beyond every buffer (all
// buffers are below 2^31 - 2^16 bytes), so a load there returns 0 and a store
// there is dropped.
constexpr int32_t OOB = 0x7FFF0000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ int32_t load_i32(__amdgpu_buffer_rsrc_t r, int32_t off) {
    return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
__device__ __forceinline__ void store_i32(__amdgpu_buffer_rsrc_t r, int32_t off, int32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v, r, off, 0, 0);
}
template <class CT>
__device__ __forceinline__ int32_t load_cost(__amdgpu_buffer_rsrc_t r, int32_t off) {
    if constexpr (sizeof(CT) == 2) return (int32_t)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    else return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// Cache policy of a buffer access that must be coherent at device scope (sc1): the
// access is performed at the level shared by all compute units of the device.
constexpr int CPOL_DEVICE = 16;

// N consecutive int32 at byte offset off (dword aligned), widest loads first; AUX is the
// cache policy.
template <int N, int AUX = 0>
__device__ __forceinline__ void load_vec(__amdgpu_buffer_rsrc_t r, int32_t off, int32_t* dst) {
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int k = 0; k < N; k += 4) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off + 4 * k, 0, AUX);
            dst[k] = (int32_t)v[0]; dst[k + 1] = (int32_t)v[1]; dst[k + 2] = (int32_t)v[2]; dst[k + 3] = (int32_t)v[3];
        }
    } else if constexpr (N == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
        dst[0] = (int32_t)v[0]; dst[1] = (int32_t)v[1];
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) dst[k] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off + 4 * k, 0, AUX);
    }
}
template <int N, int AUX = 0>
__device__ __forceinline__ void store_vec(__amdgpu_buffer_rsrc_t r, int32_t off, const int32_t* src) {
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int k = 0; k < N; k += 4) {
            const uint32_t __attribute__((ext_vector_type(4))) v = {(uint32_t)src[k], (uint32_t)src[k + 1],
                                                                    (uint32_t)src[k + 2], (uint32_t)src[k + 3]};
            __builtin_amdgcn_raw_buffer_store_b128(v, r, off + 4 * k, 0, AUX);
        }
    } else if constexpr (N == 2) {
        const uint32_t __attribute__((ext_vector_type(2))) v = {(uint32_t)src[0], (uint32_t)src[1]};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, AUX);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) __builtin_amdgcn_raw_buffer_store_b32((uint32_t)src[k], r, off + 4 * k, 0, AUX);
    }
}

// Cost element kinds: int16 one by one, int16 in aligned pairs, int32 in runs.
struct Pair16 {};
template <class CK> struct CostBytes { static constexpr int value = sizeof(CK); };
template <> struct CostBytes<Pair16> { static constexpr int value = 2; };

// N consecutive costs starting at byte offset off; OOB offsets give zeros.
// The loaded words stay packed (cost_words) until a cost is used (cost_elem):
// unpacking at the load would make the loop wait for the load where it is
// issued instead of where its value is consumed.
template <class CK, int N>
struct CostWords {
    static constexpr int value = (std::is_same<CK, Pair16>::value && N % 2 == 0) ? N / 2 : N;
};

template <class CK, int N>
__device__ __forceinline__ void load_cost_words(__amdgpu_buffer_rsrc_t r, int32_t off, int32_t* w) {
    if constexpr (sizeof(CK) == 4) {
        load_vec<N>(r, off, w);
    } else if constexpr (std::is_same<CK, Pair16>::value && N % 2 == 0) {
        load_vec<N / 2>(r, off, w);
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k)
            w[k] = (int32_t)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off + 2 * k, 0, 0);
    }
}

template <class CK, int N>
__device__ __forceinline__ int32_t cost_elem(const int32_t* w, int k) {
    if constexpr (std::is_same<CK, Pair16>::value && N % 2 == 0)
        return (k & 1) ? (w[k >> 1] >> 16) : (int32_t)(int16_t)(w[k >> 1] & 0xFFFF);
    else
        return w[k];
}

// ---- DPP (GFX9 encodings) --------------------------------------------------
constexpr int DPP_QUAD_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROW_MIRROR = 0x140;    // lane i <- 15 - i (within the row)
constexpr int DPP_HALF_MIRROR = 0x141;   // lane i <- 7 - i (within each half row)
constexpr int dpp_row_shr(int n) { return 0x110 + n; }   // lane i <- i - n, row lanes < n keep old
constexpr int dpp_row_shl(int n) { return 0x100 + n; }   // lane i <- i + n, row lanes >= 16-n keep old
constexpr int dpp_row_ror(int n) { return 0x120 + n; }   // lane i <- (i - n) mod 16

template <int CTRL>
__device__ __forceinline__ int32_t dpp(int32_t old, int32_t v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, 0xF, false);
}

// rows r <- r - 1 (r = 1, 2, 3; row 0 gets row 0)
__device__ __forceinline__ int32_t rows_up(int32_t v, int32_t lane) {
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);   // [r0 r0 r2 r2], [r1 r1 r3 r3]
    const auto b = __builtin_amdgcn_permlane32_swap(a[1], a[1], false, false);  // [r1 r1 r1 r1]
    return (lane >> 4) == 2 ? (int32_t)b[0] : (int32_t)a[0];
}
// rows r <- r + 1 (r = 0, 1, 2; row 3 gets row 3)
__device__ __forceinline__ int32_t rows_down(int32_t v, int32_t lane) {
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(a[0], a[0], false, false);  // [r2 r2 r2 r2]
    return (lane >> 4) == 1 ? (int32_t)b[1] : (int32_t)a[1];
}

// Value of lane (lane - N); lanes below N receive unspecified values.
template <int N>
__device__ __forceinline__ int32_t lanes_up(int32_t v, int32_t lane) {
    static_assert(N >= 1 && N <= 32, "shift");
    if constexpr (N == 32) {
        return (int32_t)__builtin_amdgcn_permlane32_swap(v, v, false, false)[0];
    } else if constexpr (N == 16) {
        return rows_up(v, lane);
    } else {
        const int32_t t = dpp<dpp_row_ror(N)>(v, v);
        return (lane & 15) >= N ? t : rows_up(t, lane);
    }
}
// Value of lane (lane + N); lanes at or above 64 - N receive unspecified values.
template <int N>
__device__ __forceinline__ int32_t lanes_down(int32_t v, int32_t lane) {
    static_assert(N >= 1 && N <= 32, "shift");
    if constexpr (N == 32) {
        return (int32_t)__builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
    } else if constexpr (N == 16) {
        return rows_down(v, lane);
    } else {
        const int32_t t = dpp<dpp_row_ror(16 - N)>(v, v);
        return (lane & 15) < 16 - N ? t : rows_down(t, lane);
    }
}
// ---- lines of NL lanes, STEP lanes apart ------------------------------------
// pos is the lane's index along its line.  Lines of x (STEP = 1) lie in one
// lane row when NL <= 16; lines of y (STEP = PX) fill whole rows.

// value at position pos - D of the line; own value when pos < D
template <int NL, int STEP, int D>
__device__ __forceinline__ int32_t line_up(int32_t v, int32_t pos, int32_t lane) {
    constexpr int n = D * STEP;
    if constexpr (NL * STEP <= 16) {
        const int32_t r = dpp<dpp_row_shr(n)>(v, v);
        if constexpr (NL * STEP == 16) return r;
        else return pos >= D ? r : v;
    } else {
        const int32_t r = lanes_up<n>(v, lane);
        return pos >= D ? r : v;
    }
}
// value at position pos + D of the line; own value when pos + D >= NL
template <int NL, int STEP, int D>
__device__ __forceinline__ int32_t line_down(int32_t v, int32_t pos, int32_t lane) {
    constexpr int n = D * STEP;
    if constexpr (NL * STEP <= 16) {
        const int32_t r = dpp<dpp_row_shl(n)>(v, v);
        if constexpr (NL * STEP == 16) return r;
        else return pos + D < NL ? r : v;
    } else {
        const int32_t r = lanes_down<n>(v, lane);
        return pos + D < NL ? r : v;
    }
}
// minimum over the NL lanes of the line
template <int NL, int STEP>
__device__ __forceinline__ int32_t line_min(int32_t v, int32_t lane) {
    auto mx = [](int32_t x, int32_t y) { return imin(x, y); };
    if constexpr (NL == 1) {
        return v;
    } else if constexpr (NL * STEP < 16) {
        static_assert(STEP == 1, "short lines must run along x");
        v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_QUAD_XOR1, 0xF, 0xF, false));
        if constexpr (NL >= 4) v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_QUAD_XOR2, 0xF, 0xF, false));
        if constexpr (NL >= 8) v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_HALF_MIRROR, 0xF, 0xF, false));
        return v;
    } else {
        // inside a row the line's lanes form a coset of the rotation by STEP
        if constexpr (STEP == 1) {
            v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_QUAD_XOR1, 0xF, 0xF, false));
            v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_QUAD_XOR2, 0xF, 0xF, false));
            v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_HALF_MIRROR, 0xF, 0xF, false));
            v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, DPP_ROW_MIRROR, 0xF, 0xF, false));
        } else {
            if constexpr (STEP <= 2) v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, dpp_row_ror(2), 0xF, 0xF, false));
            if constexpr (STEP <= 4) v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, dpp_row_ror(4), 0xF, 0xF, false));
            if constexpr (STEP <= 8) v = mx(v, __builtin_amdgcn_update_dpp(0x7FFFFFFF, v, dpp_row_ror(8), 0xF, 0xF, false));
        }
        // across rows: the lanes 16 and 32 apart, one ds_bpermute each
        if constexpr (NL * STEP >= 32) v = mx(v, __builtin_amdgcn_ds_bpermute((lane ^ 16) * 4, v));
        if constexpr (NL * STEP >= 64) v = mx(v, __builtin_amdgcn_ds_bpermute((lane ^ 32) * 4, v));
        return v;
    }
}

// ---- fused min-scans ---------------------------------------------------------
// dpp<...>(IDENT, v) reads IDENT where the source lane lies outside the row or
// outside the enabled banks; min(x, that) then compiles to one v_min_i32_dpp.
constexpr int32_t IDENT = 0x7FFFFFFF;
constexpr int DPP_QP_SHR1 = 0x90;        // quad_perm [0,0,1,2]: lane i <- i-1 (lane 0 <- 0)
constexpr int DPP_QP_SHR2 = 0x44;        // quad_perm [0,1,0,1]: lane i <- i-2 (lanes 0,1 <- self)
constexpr int DPP_QP_SHL1 = 0xF9;        // quad_perm [1,2,3,3]: lane i <- i+1 (lane 3 <- 3)
constexpr int DPP_QP_SHL2 = 0xEE;        // quad_perm [2,3,2,3]: lane i <- i+2 (lanes 2,3 <- self)
constexpr int DPP_QP_BC3 = 0xFF;         // quad_perm [3,3,3,3]
constexpr int DPP_QP_BC0 = 0x00;         // quad_perm [0,0,0,0]
constexpr int DPP_QP_PAIR_SHR = 0xA0;    // quad_perm [0,0,2,2]: odd lanes <- even neighbour
constexpr int DPP_QP_PAIR_SHL = 0xF5;    // quad_perm [1,1,3,3]: even lanes <- odd neighbour

template <int CTRL, int BANKS = 0xF>
__device__ __forceinline__ int32_t minx(int32_t x, int32_t src) {
    return imin(x, __builtin_amdgcn_update_dpp(IDENT, src, CTRL, 0xF, BANKS, false));
}

// Inclusive prefix minimum along the line (positions 0..pos).
template <int NL, int STEP>
__device__ __forceinline__ int32_t scan_up(int32_t v, int32_t pos, int32_t lane) {
    if constexpr (NL == 1) {
        return v;
    } else if constexpr (STEP == 1 && NL == 2) {
        return minx<DPP_QP_PAIR_SHR>(v, v);
    } else if constexpr (STEP == 1 && NL == 4) {
        v = minx<DPP_QP_SHR1>(v, v);
        return minx<DPP_QP_SHR2>(v, v);
    } else if constexpr (STEP == 1 && NL == 8) {
        v = minx<DPP_QP_SHR1>(v, v);
        v = minx<DPP_QP_SHR2>(v, v);
        const int32_t t = dpp<DPP_QP_BC3>(v, v);          // quad totals
        return minx<dpp_row_shr(4), 0xA>(v, t);          // banks 1, 3 take the quad below
    } else if constexpr (NL * STEP == 16) {
        if constexpr (NL > 1) v = minx<dpp_row_shr(STEP)>(v, v);
        if constexpr (NL > 2) v = minx<dpp_row_shr(2 * STEP)>(v, v);
        if constexpr (NL > 4) v = minx<dpp_row_shr(4 * STEP)>(v, v);
        if constexpr (NL > 8) v = minx<dpp_row_shr(8 * STEP)>(v, v);
        return v;
    } else {
        // the line crosses 16-lane rows
        if constexpr (NL > 1) v = imin(v, line_up<NL, STEP, 1>(v, pos, lane));
        if constexpr (NL > 2) v = imin(v, line_up<NL, STEP, 2>(v, pos, lane));
        if constexpr (NL > 4) v = imin(v, line_up<NL, STEP, 4>(v, pos, lane));
        if constexpr (NL > 8) v = imin(v, line_up<NL, STEP, 8>(v, pos, lane));
        if constexpr (NL > 16) v = imin(v, line_up<NL, STEP, 16>(v, pos, lane));
        if constexpr (NL > 32) v = imin(v, line_up<NL, STEP, 32>(v, pos, lane));
        return v;
    }
}

// Inclusive suffix minimum along the line (positions pos..NL-1).
template <int NL, int STEP>
__device__ __forceinline__ int32_t scan_down(int32_t v, int32_t pos, int32_t lane) {
    if constexpr (NL == 1) {
        return v;
    } else if constexpr (STEP == 1 && NL == 2) {
        return minx<DPP_QP_PAIR_SHL>(v, v);
    } else if constexpr (STEP == 1 && NL == 4) {
        v = minx<DPP_QP_SHL1>(v, v);
        return minx<DPP_QP_SHL2>(v, v);
    } else if constexpr (STEP == 1 && NL == 8) {
        v = minx<DPP_QP_SHL1>(v, v);
        v = minx<DPP_QP_SHL2>(v, v);
        const int32_t t = dpp<DPP_QP_BC0>(v, v);          // quad totals (from the top)
        return minx<dpp_row_shl(4), 0x5>(v, t);          // banks 0, 2 take the quad above
    } else if constexpr (NL * STEP == 16) {
        if constexpr (NL > 1) v = minx<dpp_row_shl(STEP)>(v, v);
        if constexpr (NL > 2) v = minx<dpp_row_shl(2 * STEP)>(v, v);
        if constexpr (NL > 4) v = minx<dpp_row_shl(4 * STEP)>(v, v);
        if constexpr (NL > 8) v = minx<dpp_row_shl(8 * STEP)>(v, v);
        return v;
    } else {
        if constexpr (NL > 1) v = imin(v, line_down<NL, STEP, 1>(v, pos, lane));
        if constexpr (NL > 2) v = imin(v, line_down<NL, STEP, 2>(v, pos, lane));
        if constexpr (NL > 4) v = imin(v, line_down<NL, STEP, 4>(v, pos, lane));
        if constexpr (NL > 8) v = imin(v, line_down<NL, STEP, 8>(v, pos, lane));
        if constexpr (NL > 16) v = imin(v, line_down<NL, STEP, 16>(v, pos, lane));
        if constexpr (NL > 32) v = imin(v, line_down<NL, STEP, 32>(v, pos, lane));
        return v;
    }
}

// Value at position pos - 1 of the line, FILL at position 0.
template <int NL, int STEP, int32_t FILL = IDENT>
__device__ __forceinline__ int32_t carry_up(int32_t v, int32_t pos, int32_t lane) {
    if constexpr (NL * STEP == 16) {
        return __builtin_amdgcn_update_dpp(FILL, v, dpp_row_shr(STEP), 0xF, 0xF, false);
    } else if constexpr (NL * STEP < 16) {
        const int32_t r = __builtin_amdgcn_update_dpp(FILL, v, dpp_row_shr(STEP), 0xF, 0xF, false);
        return pos == 0 ? FILL : r;
    } else {
        const int32_t r = lanes_up<STEP>(v, lane);
        return pos == 0 ? FILL : r;
    }
}
// Value at position pos + 1 of the line, FILL at position NL - 1.
template <int NL, int STEP, int32_t FILL = IDENT>
__device__ __forceinline__ int32_t carry_down(int32_t v, int32_t pos, int32_t lane) {
    if constexpr (NL * STEP == 16) {
        return __builtin_amdgcn_update_dpp(FILL, v, dpp_row_shl(STEP), 0xF, 0xF, false);
    } else if constexpr (NL * STEP < 16) {
        const int32_t r = __builtin_amdgcn_update_dpp(FILL, v, dpp_row_shl(STEP), 0xF, 0xF, false);
        return pos == NL - 1 ? FILL : r;
    } else {
        const int32_t r = lanes_down<STEP>(v, lane);
        return pos == NL - 1 ? FILL : r;
    }
}

// ---- linear RMS on one dimension -------------------------------------------
// For every line along the dimension: the L1 distance transform
//   L(v) = min_v' h(v') + lam |v - v'|
// i.e. the forward pass of eq. L_dec3 and the backward pass of eq. L_dec5,
// then the clip min(L, line_min + clipd) when clip is set (per-dimension
// truncation).  Lines are split over NL lanes, K labels per lane.  The passes
// run on g(v) = h(v) - lam v (forward) and h(v) + lam v (backward), where the
// recursions become plain prefix / suffix minima:
//   min_{v' <= v} h(v') + lam (v - v') = lam v + min_{v' <= v} g(v').
// lv[k] = lam * (index of label k along the line).  Returns min h of the line.
template <int NL, int K, int STEP>
__device__ __forceinline__ int32_t l1_line(int32_t (&val)[K], const int32_t (&lv)[K], const int32_t clipd,
                                           const bool clip, const int32_t pos, const int32_t lane) {
    int32_t p[K], q[K];
    p[0] = val[0] - lv[0];
#pragma unroll
    for (int k = 1; k < K; ++k) p[k] = imin(p[k - 1], val[k] - lv[k]);
    q[K - 1] = val[K - 1] + lv[K - 1];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) q[k] = imin(q[k + 1], val[k] + lv[k]);
    int32_t m = val[0];
#pragma unroll
    for (int k = 1; k < K; ++k) m = imin(m, val[k]);
    if constexpr (NL > 1) {
        const int32_t tf = scan_up<NL, STEP>(p[K - 1], pos, lane);
        const int32_t tb = scan_down<NL, STEP>(q[0], pos, lane);
        const int32_t cf = carry_up<NL, STEP>(tf, pos, lane);
        const int32_t cb = carry_down<NL, STEP>(tb, pos, lane);
        m = line_min<NL, STEP>(m, lane);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            p[k] = imin(p[k], cf);
            q[k] = imin(q[k], cb);
        }
    }
    const int32_t cap = clip ? m + clipd : IDENT;
#pragma unroll
    for (int k = 0; k < K; ++k) val[k] = imin3(p[k] + lv[k], q[k] - lv[k], cap);
    return m;
}

// ---- general RMS on one dimension ------------------------------------------------
// For every line along the dimension: the window minimum of eq. M_decmp1 with
// the penalty inside the minimum,
//   W(v) = min_{|u| < g} h(v - u) + lam f(u),
// then the clip min(W, line_min + clipd) when clip is set (clipd = lam f(g)).
// It is exact for any increasing f; here f(u) = u (truncated linear prior) or
// u^2 (truncated squared prior).  A line of n labels takes nw = min(g, n) - 1
// window steps on each side.  On packed keys lam is the penalty unit shifted
// above the index bits.
//
// Two ways, chosen per kernel so that the step has no branch:
//   short windows (nw <= 2, which covers g <= 3, the paper's setups): the values
//     of the labels up to two positions below and above are fetched a whole
//     lane at a time (one cross-lane move per register and lane hop, PADV past
//     the ends of the line), so the moves are independent of each other, and
//     each label takes two three-way minima; a step outside the window gets the
//     penalty PEN_OFF, which no candidate survives.  For the linear prior with
//     g <= 3 this is cheaper than the two recursions of the linear RMS;
//   any window (squared prior): the window is walked one label at a time: after
//     u steps up[k] holds the value u labels below label k and dn[k] the value
//     u labels above.

// Penalty of a window step outside the window: above every real value, and PADV plus it
// still fits in int32.
constexpr int32_t PEN_OFF = 0x40000000;

// Window steps and the penalties lam f(u) of the first two (u = 1, 2) along x, y and z.
struct WinPen {
    int32_t lam, nwx, nwy, nwz;
    int32_t px[2], py[2], pz[2];
    __device__ __forceinline__ WinPen(const int32_t lam_, const int32_t g, const int32_t qx, const int32_t qy,
                                      const bool squared, const int32_t qz = 1) {
        lam = lam_;
        nwx = min(g, qx) - 1;
        nwy = min(g, qy) - 1;
        nwz = min(g, qz) - 1;
#pragma unroll
        for (int u = 1; u <= 2; ++u) {
            const int32_t p = lam * (squared ? u * u : u);
            px[u - 1] = u <= nwx ? p : PEN_OFF;
            py[u - 1] = u <= nwy ? p : PEN_OFF;
            pz[u - 1] = u <= nwz ? p : PEN_OFF;
        }
    }
};

template <int NL, int K, int STEP, int NW>
__device__ __forceinline__ void quad_window(int32_t (&val)[K], const int32_t* pen, const int32_t pos,
                                            const int32_t lane) {
    constexpr int HOPS = (NW + K - 1) / K;
    int32_t lo[HOPS + 1][K], hi[HOPS + 1][K];    // [h][k]: the label h lanes below / above label k
#pragma unroll
    for (int k = 0; k < K; ++k) {
        lo[0][k] = val[k];
        hi[0][k] = val[k];
    }
#pragma unroll
    for (int h = 1; h <= HOPS; ++h)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if constexpr (NL * STEP > 16) {
                // lines across 16-lane rows: one ds_bpermute per move (the permlane route
                // takes a DPP rotation, two swaps and selects)
                const int32_t u = __builtin_amdgcn_ds_bpermute((lane - STEP) * 4, lo[h - 1][k]);
                const int32_t d = __builtin_amdgcn_ds_bpermute((lane + STEP) * 4, hi[h - 1][k]);
                lo[h][k] = pos == 0 ? PADV : u;
                hi[h][k] = pos == NL - 1 ? PADV : d;
            } else if constexpr (NL > 1) {
                lo[h][k] = carry_up<NL, STEP, PADV>(lo[h - 1][k], pos, lane);
                hi[h][k] = carry_down<NL, STEP, PADV>(hi[h - 1][k], pos, lane);
            } else {
                lo[h][k] = PADV;
                hi[h][k] = PADV;
            }
        }
    int32_t out[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int32_t o = val[k];
#pragma unroll
        for (int u = 1; u <= NW; ++u) {
            const int jl = k - u, jh = k + u;           // lane-local label indexes
            const int hl = jl >= 0 ? 0 : (K - 1 - jl) / K, hh = jh / K;
            o = imin3(o, lo[hl][jl + hl * K] + pen[u - 1], hi[hh][jh - hh * K] + pen[u - 1]);
        }
        out[k] = o;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) val[k] = out[k];
}

// squared prior only: lam u^2 accumulates as the sum of lam (2i - 1)
template <int NL, int K, int STEP>
__device__ __forceinline__ void quad_walk(int32_t (&val)[K], const int32_t lam, const int32_t nw,
                                          const int32_t pos, const int32_t lane) {
    int32_t up[K], dn[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        up[k] = val[k];
        dn[k] = val[k];
    }
    int32_t pen = 0, inc = lam;
    for (int32_t u = 0; u < nw; ++u) {
        pen += inc;
        inc += 2 * lam;
        int32_t cu = PADV, cd = PADV;
        if constexpr (NL > 1) {
            cu = carry_up<NL, STEP, PADV>(up[K - 1], pos, lane);
            cd = carry_down<NL, STEP, PADV>(dn[0], pos, lane);
        }
#pragma unroll
        for (int k = K - 1; k > 0; --k) up[k] = up[k - 1];
        up[0] = cu;
#pragma unroll
        for (int k = 0; k < K - 1; ++k) dn[k] = dn[k + 1];
        dn[K - 1] = cd;
#pragma unroll
        for (int k = 0; k < K; ++k) val[k] = imin3(val[k], up[k] + pen, dn[k] + pen);
    }
}

// NWK 1 or 2: nw <= NWK with the step penalties pen; NWK 0: any nw walked, squared prior.
// Returns min h of the line.
template <int NL, int K, int STEP, int NWK>
__device__ __forceinline__ int32_t window_line(int32_t (&val)[K], const int32_t (&pen)[2], const int32_t lam,
                                             const int32_t nw, const int32_t clipd, const bool clip,
                                             const int32_t pos, const int32_t lane) {
    int32_t m = val[0];
#pragma unroll
    for (int k = 1; k < K; ++k) m = imin(m, val[k]);
    if constexpr (NL > 1) m = line_min<NL, STEP>(m, lane);
    if constexpr (NWK == 0) quad_walk<NL, K, STEP>(val, lam, nw, pos, lane);
    else quad_window<NL, K, STEP, NWK>(val, pen, pos, lane);
    if (clip) {
#pragma unroll
        for (int k = 0; k < K; ++k) val[k] = imin(val[k], m + clipd);
    }
    return m;
}

// ---- minimum search between shifted label frames -----------------------------
// The label-window solve keeps every vertex's labels in a frame of its own; the
// sum handed to a neighbour is evaluated in the neighbour's frame, shifted by d
// labels along the line.  With source labels i = 0..n-1 (n = NL K) and target
// labels j (source position j + d):
//   out(j) = min_i val(i) + lam |j + d - i|, clipped at (line min + clipd)
// which is the L1 transform of l1_line read at the shifted position, with the
// exact continuation outside the source range:
//   forward part  min_{i <= s} g(i) + lam s      (s = j + d >= 0; s > n-1 takes all i)
//   backward part min_{i >= s} (val(i) + lam i) - lam s   (s <= n-1; s < 0 takes all i)
// The shifted reads go through a per-wavefront LDS area sp / sq of 64 K ints.
template <int NL, int K, int STEP>
__device__ __forceinline__ int32_t l1_line_shift(int32_t (&val)[K], const int32_t lam, const int32_t clipd,
                                                 const bool clip, const int32_t pos, const int32_t lane,
                                                 const int32_t d, int32_t* sp, int32_t* sq) {
    int32_t p[K], q[K];
    p[0] = val[0] - lam * (pos * K);
#pragma unroll
    for (int k = 1; k < K; ++k) p[k] = imin(p[k - 1], val[k] - lam * (pos * K + k));
    q[K - 1] = val[K - 1] + lam * (pos * K + K - 1);
#pragma unroll
    for (int k = K - 2; k >= 0; --k) q[k] = imin(q[k + 1], val[k] + lam * (pos * K + k));
    int32_t m = val[0];
#pragma unroll
    for (int k = 1; k < K; ++k) m = imin(m, val[k]);
    if constexpr (NL > 1) {
        const int32_t tf = scan_up<NL, STEP>(p[K - 1], pos, lane);
        const int32_t tb = scan_down<NL, STEP>(q[0], pos, lane);
        const int32_t cf = carry_up<NL, STEP>(tf, pos, lane);
        const int32_t cb = carry_down<NL, STEP>(tb, pos, lane);
        m = line_min<NL, STEP>(m, lane);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            p[k] = imin(p[k], cf);
            q[k] = imin(q[k], cb);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        sp[lane * K + k] = p[k];
        sq[lane * K + k] = q[k];
    }
    constexpr int32_t n = NL * K;
    const int32_t cap = clip ? m + clipd : IDENT;
    const int32_t base = lane - pos * STEP;           // lane of position 0 of this line
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int32_t s = pos * K + k + d;
        const int32_t sf = s < n - 1 ? s : n - 1;
        const int32_t sb = s > 0 ? s : 0;
        const int32_t af = (base + (sf >= 0 ? sf : 0) / K * STEP) * K + (sf >= 0 ? sf : 0) % K;
        const int32_t ab = (base + (sb < n ? sb : n - 1) / K * STEP) * K + (sb < n ? sb : n - 1) % K;
        const int32_t vf = sp[af] + lam * s;
        const int32_t vb = sq[ab] - lam * s;
        val[k] = imin3(s >= 0 ? vf : IDENT, s <= n - 1 ? vb : IDENT, cap);
    }
    return m;
}

// The same between shifted frames with the general RMS window (one label per lane, windows of
// at most two steps per side): target label j takes the source labels i = j + d - u, |u| <= nw,
// that lie in the source frame, each plus lam |u|, read from their lanes with ds_bpermute (the
// five reads are independent of each other), then the clip.  Source labels outside the frame
// do not exist for the neighbour, as in l1_line_shift.  Returns min val of the line.
template <int NL, int STEP>
__device__ __forceinline__ int32_t window_line_shift(int32_t& val, const int32_t (&pen)[2], const int32_t nw,
                                                     const int32_t clipd, const bool clip, const int32_t pos,
                                                     const int32_t lane, const int32_t d) {
    const int32_t m = line_min<NL, STEP>(val, lane);
    const int32_t base = lane - pos * STEP;           // lane of position 0 of this line
    const int32_t s = pos + d;
    // a target with no source label in its window keeps PADV, which the next dimension's
    // penalties cannot carry past int32 (joint truncation clips only at the end)
    int32_t o = PADV;
#pragma unroll
    for (int u = -2; u <= 2; ++u) {
        const int32_t i = s - u;
        const int au = u < 0 ? -u : u;
        const bool ok = (uint32_t)i < (uint32_t)NL && au <= nw;
        const int32_t v = __builtin_amdgcn_ds_bpermute((base + (ok ? i : 0) * STEP) * 4, val);
        const int32_t c = au == 0 ? v : v + pen[au - 1];
        o = ok ? imin(o, c) : o;
    }
    val = clip ? imin(o, m + clipd) : o;
    return m;
}

// M between shifted frames by the general RMS window, for tiles of one label per lane;
// nw = T - 1 <= 2 (the frame is the source's whole label range).  Same contract as
// min_search_shift.
template <class T>
__device__ __forceinline__ void min_search_shift_window(int32_t (&h)[T::KY][T::KX], const WinPen& wp,
                                                        const int32_t clipd, const bool joint, const int32_t lane,
                                                        const int32_t dx, const int32_t dy) {
    static_assert(T::KX == 1 && T::KY == 1, "one label per lane");
    const int32_t l = lane % T::G;
    const int32_t px = l % T::PX, py = l / T::PX;
    const int32_t rowmin = window_line_shift<T::PX, 1>(h[0][0], wp.px, wp.nwx, clipd, !joint, px, lane, dx);
    int32_t gmin = rowmin;
    if constexpr (T::PY > 1) gmin = line_min<T::PY, T::PX>(gmin, lane);
    window_line_shift<T::PY, T::PX>(h[0][0], wp.py, wp.nwy, clipd, !joint, py, lane, dy);
    if (joint) h[0][0] = imin(h[0][0], gmin + clipd);
}

// Minimum of v over the G lanes of this lane's group.
template <class T>
__device__ __forceinline__ int32_t group_min(int32_t v, const int32_t lane) {
    v = line_min<T::PX, 1>(v, lane);
    if constexpr (T::PY > 1) v = line_min<T::PY, T::PX>(v, lane);
    return v;
}

// Distance offsets of the lane's labels along x, y and z: lam * vx, lam * vy and lam * vz.
template <class T>
struct LineIndex {
    int32_t lx[T::KX], ly[T::KY], lz[T::KZ];
    __device__ __forceinline__ LineIndex(const int32_t lam, const int32_t lane) {
        const int32_t l = lane % T::G;
        const int32_t px = l % T::PX, py = l / T::PX;
#pragma unroll
        for (int k = 0; k < T::KX; ++k) lx[k] = lam * (px * T::KX + k);
#pragma unroll
        for (int k = 0; k < T::KY; ++k) ly[k] = lam * (py * T::KY + k);
#pragma unroll
        for (int k = 0; k < T::KZ; ++k) lz[k] = lam * k;
    }
};

// The minimum search operator M (Sec. 2 eq. M_strf) for the truncated linear
// prior, computed by the linear RMS of Sec. 3.2:
//   joint == false (per-dimension truncation): each label dimension r gets the
//     L1 transform of its lines clipped at (line minimum + clipd), the
//     decomposition of eq. derivation2 applied per dimension;
//   joint == true (truncation of the summed distance, the paper's prior):
//     L_z(L_y(L_x(h))) clipped at (min h + clipd), eq. L_dec7.
// h holds the lane's KR rows of KX labels; padding labels must hold PADV on entry.
// The dimensions run x, y, z: a padding plane of z (vz >= qz) is all PADV until the z
// operator, so it never reaches a real label.  Returns min h over the whole vertex.
template <class T>
__device__ __forceinline__ int32_t min_search(int32_t (&h)[T::KR][T::KX], const LineIndex<T>& li,
                                              const int32_t clipd, const bool joint, const int32_t lane) {
    const int32_t l = lane % T::G;
    const int32_t px = l % T::PX, py = l / T::PX;
    constexpr bool one_dim = T::PY * T::KY == 1 && T::KZ == 1;
    int32_t rowmin = PADV;
#pragma unroll
    for (int r = 0; r < T::KR; ++r) {
        // with a single label dimension the final clip is the per-line clip
        const int32_t lm = l1_line<T::PX, T::KX, 1>(h[r], li.lx, clipd, !joint || one_dim, px, lane);
        rowmin = imin(rowmin, lm);
    }
    if constexpr (one_dim) {
        return rowmin;
    } else {
        int32_t gmin = rowmin;
        if constexpr (T::PY > 1) gmin = line_min<T::PY, T::PX>(gmin, lane);
        if constexpr (T::PY * T::KY > 1) {
#pragma unroll
            for (int kz = 0; kz < T::KZ; ++kz)
#pragma unroll
                for (int kx = 0; kx < T::KX; ++kx) {
                    int32_t col[T::KY];
#pragma unroll
                    for (int ky = 0; ky < T::KY; ++ky) col[ky] = h[kz * T::KY + ky][kx];
                    l1_line<T::PY, T::KY, T::PX>(col, li.ly, clipd, !joint, py, lane);
#pragma unroll
                    for (int ky = 0; ky < T::KY; ++ky) h[kz * T::KY + ky][kx] = col[ky];
                }
        }
        if constexpr (T::KZ > 1) {
#pragma unroll
            for (int ky = 0; ky < T::KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < T::KX; ++kx) {
                    int32_t zl[T::KZ];
#pragma unroll
                    for (int kz = 0; kz < T::KZ; ++kz) zl[kz] = h[kz * T::KY + ky][kx];
                    l1_line<1, T::KZ, 1>(zl, li.lz, clipd, !joint, 0, lane);
#pragma unroll
                    for (int kz = 0; kz < T::KZ; ++kz) h[kz * T::KY + ky][kx] = zl[kz];
                }
        }
        if (joint) {
#pragma unroll
            for (int r = 0; r < T::KR; ++r)
#pragma unroll
                for (int kx = 0; kx < T::KX; ++kx) h[r][kx] = imin(h[r][kx], gmin + clipd);
        }
        return gmin;
    }
}

// The windows along x and y of min_search_window (each of the lane's KZ slices of a tile of a
// three-dimensional label space); the clips per line unless joint.  Returns min h over the
// wavefront's labels.
template <class T, int NWK>
__device__ __forceinline__ int32_t min_search_xy(int32_t (&h)[T::KR][T::KX], const WinPen& sp, const int32_t clipd,
                                                 const bool joint, const int32_t lane) {
    const int32_t l = lane % T::G;
    const int32_t px = l % T::PX, py = l / T::PX;
    constexpr bool one_dim = T::PY * T::KY == 1 && T::KZ == 1;
    int32_t rowmin = PADV;
#pragma unroll
    for (int r = 0; r < T::KR; ++r) {
        const int32_t lm = window_line<T::PX, T::KX, 1, NWK>(h[r], sp.px, sp.lam, sp.nwx, clipd, !joint || one_dim,
                                                             px, lane);
        rowmin = imin(rowmin, lm);
    }
    int32_t gmin = rowmin;
    if constexpr (!one_dim) {
        if constexpr (T::PY > 1) gmin = line_min<T::PY, T::PX>(gmin, lane);
        if constexpr (T::PY * T::KY > 1) {
#pragma unroll
            for (int kz = 0; kz < T::KZ; ++kz)
#pragma unroll
                for (int kx = 0; kx < T::KX; ++kx) {
                    int32_t col[T::KY];
#pragma unroll
                    for (int ky = 0; ky < T::KY; ++ky) col[ky] = h[kz * T::KY + ky][kx];
                    window_line<T::PY, T::KY, T::PX, NWK>(col, sp.py, sp.lam, sp.nwy, clipd, !joint, py, lane);
#pragma unroll
                    for (int ky = 0; ky < T::KY; ++ky) h[kz * T::KY + ky][kx] = col[ky];
                }
        }
    }
    return gmin;
}

// The minimum search operator M computed by the general RMS of Sec. 3.1: one
// window operator per label dimension (eq. M_decmp1), clipped per line
// (per-dimension truncation) or once at (min h + clipd) (joint truncation,
// eq. M_decmp).  NWK as for window_line.  Same contract as min_search.
template <class T, int NWK>
__device__ __forceinline__ int32_t min_search_window(int32_t (&h)[T::KR][T::KX], const WinPen& sp,
                                                   const int32_t clipd, const bool joint, const int32_t lane) {
    constexpr bool one_dim = T::PY * T::KY == 1 && T::KZ == 1;
    const int32_t gmin = min_search_xy<T, NWK>(h, sp, clipd, joint, lane);
    if constexpr (one_dim) {
        return gmin;
    } else {
        if constexpr (T::KZ > 1) {
#pragma unroll
            for (int ky = 0; ky < T::KY; ++ky)
#pragma unroll
                for (int kx = 0; kx < T::KX; ++kx) {
                    int32_t zl[T::KZ];
#pragma unroll
                    for (int kz = 0; kz < T::KZ; ++kz) zl[kz] = h[kz * T::KY + ky][kx];
                    window_line<1, T::KZ, 1, NWK>(zl, sp.pz, sp.lam, sp.nwz, clipd, !joint, 0, lane);
#pragma unroll
                    for (int kz = 0; kz < T::KZ; ++kz) h[kz * T::KY + ky][kx] = zl[kz];
                }
        }
        if (joint) {
#pragma unroll
            for (int r = 0; r < T::KR; ++r)
#pragma unroll
                for (int kx = 0; kx < T::KX; ++kx) h[r][kx] = imin(h[r][kx], gmin + clipd);
        }
        return gmin;
    }
}

// M between shifted frames (see l1_line_shift): h in the source frame, the
// result in the frame shifted by (dx, dy) labels.  scratch: this wavefront's
// LDS area of 2 * 64 * max(KX, KY) ints.
template <class T>
__device__ __forceinline__ void min_search_shift(int32_t (&h)[T::KY][T::KX], const int32_t lam, const int32_t clipd,
                                                 const bool joint, const int32_t lane, const int32_t dx,
                                                 const int32_t dy, int32_t* scratch) {
    constexpr int KM = T::KX > T::KY ? T::KX : T::KY;
    int32_t* sp = scratch;
    int32_t* sq = scratch + 64 * KM;
    const int32_t l = lane % T::G;
    const int32_t px = l % T::PX, py = l / T::PX;
    int32_t rowmin = PADV;
#pragma unroll
    for (int ky = 0; ky < T::KY; ++ky)
        rowmin = imin(rowmin, l1_line_shift<T::PX, T::KX, 1>(h[ky], lam, clipd, !joint, px, lane, dx, sp, sq));
    int32_t gmin = rowmin;
    if constexpr (T::PY > 1) gmin = line_min<T::PY, T::PX>(gmin, lane);
#pragma unroll
    for (int kx = 0; kx < T::KX; ++kx) {
        int32_t col[T::KY];
#pragma unroll
        for (int ky = 0; ky < T::KY; ++ky) col[ky] = h[ky][kx];
        l1_line_shift<T::PY, T::KY, T::PX>(col, lam, clipd, !joint, py, lane, dy, sp, sq);
#pragma unroll
        for (int ky = 0; ky < T::KY; ++ky) h[ky][kx] = col[ky];
    }
    if (joint) {
#pragma unroll
        for (int ky = 0; ky < T::KY; ++ky)
#pragma unroll
            for (int kx = 0; kx < T::KX; ++kx) h[ky][kx] = imin(h[ky][kx], gmin + clipd);
    }
}

}  // namespace edp
