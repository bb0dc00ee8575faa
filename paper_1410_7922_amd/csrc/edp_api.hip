// C ABI of the gfx950 scanline-DP / EDP library: argument checks, workspace
// layout and the order of kernel launches (Mozerov, arXiv 1410.7922,
// Algorithm 1 for edp_solve, Sec. 2 eq. base and Sec. 4.1 for the DP).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>

#include "../../include/edp.h"
#include "edp_internal.hpp"

namespace edp {

namespace {

const TileShape kTiles[NUM_TILES] = {
#define EDP_ROW(id, px, kx, py, ky) {px, kx, py, ky},
    EDP_TILE_LIST(EDP_ROW)
#undef EDP_ROW
};

constexpr size_t kAlign = 256;
size_t up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

int qt_of(int tile) {
    const TileShape& t = kTiles[tile];
    return t.px * t.py * t.kx * t.ky;
}
int group_of(int tile) { return kTiles[tile].px * kTiles[tile].py; }
int elems_of(int tile) { return kTiles[tile].kx * kTiles[tile].ky; }

bool fits(int tile, int qx, int qy) {
    const TileShape& t = kTiles[tile];
    return t.px * t.kx >= qx && t.py * t.ky >= qy;
}

// Built-in choice: least padding; then vertices that fill one 16-lane row
// (every cross-lane step of the minimum search is a single DPP instruction);
// then fewest labels per lane.
int auto_tile(int qx, int qy) {
    int best = -1;
    auto score = [](int t) { return (group_of(t) == 16 ? 0 : 1000) + elems_of(t); };
    for (int t = 0; t < NUM_TILES; ++t) {
        if (!fits(t, qx, qy)) continue;
        if (best < 0 || qt_of(t) < qt_of(best) || (qt_of(t) == qt_of(best) && score(t) < score(best))) best = t;
    }
    return best;
}

int ibits_of(int q) {
    int b = 1;
    while ((1 << b) < q) ++b;
    return b;
}

int64_t cost_bound_of(const edp_problem* p) {
    if (p->cost_bound > 0) return p->cost_bound;
    return p->dtype == EDP_I16 ? 32768 : -1;
}

int64_t vmax_of(const edp_problem* p) {
    const int64_t dims = (p->trunc_mode == EDP_TRUNC_PER_DIM && p->qy > 1) ? 2 : 1;
    return (int64_t)p->lambda * p->trunc * dims;
}

edp_status check_problem(const edp_problem* p, int op) {
    if (!p) return EDP_E_INVALID;
    if (p->width < 1 || p->height < 1 || p->qx < 1 || p->qy < 1) return EDP_E_INVALID;
    if ((int64_t)p->width * p->height > (int64_t)1 << 30) return EDP_E_INVALID;
    if ((int64_t)p->qx * p->qy > 4096) return EDP_E_INVALID;
    if (p->dtype != EDP_I16 && p->dtype != EDP_I32) return EDP_E_INVALID;
    if (p->trunc_mode != EDP_TRUNC_PER_DIM && p->trunc_mode != EDP_TRUNC_JOINT) return EDP_E_INVALID;
    if (p->lambda < 0 || p->lambda > 65535 || p->trunc < 1 || p->trunc > 4096) return EDP_E_INVALID;
    if (p->cost_bound < 0) return EDP_E_INVALID;
    if (op == EDP_OP_EDP) {
        if (p->iterations < 1 || p->iterations > 4096) return EDP_E_INVALID;
        if ((int64_t)4 * p->iterations * ((int64_t)p->width + 1) >= ((int64_t)1 << 31)) return EDP_E_INVALID;
    }
    const int64_t b = cost_bound_of(p);
    if (b < 0) return EDP_E_INVALID;  // int32 costs need a declared bound
    if (op == EDP_OP_EDP) {
        // empirical int32 guard for the EDP sums (they grow with the grid extent)
        if ((int64_t)(p->width + p->height) * (b + 4 * vmax_of(p)) * 8 >= ((int64_t)1 << 29)) return EDP_E_RANGE;
    } else {
        const int64_t q = (int64_t)p->qx * p->qy;
        const int64_t span = b + vmax_of(p) + (int64_t)p->lambda * (p->qx + p->qy + 64);
        if ((span << ibits_of((int)q)) >= ((int64_t)1 << 28)) return EDP_E_RANGE;
    }
    return EDP_OK;
}

edp_status pick_tile(const edp_problem* p, const edp_tuning* tu, int* tile) {
    int t = (tu && tu->tile >= 0) ? tu->tile : auto_tile(p->qx, p->qy);
    if (t < 0) return EDP_E_UNSUPPORTED;
    if (t >= NUM_TILES || !fits(t, p->qx, p->qy)) return EDP_E_INVALID;
    *tile = t;
    return EDP_OK;
}

struct Launch {
    int tile, split, waves, chunk, ring;
    int rpw;            // scanlines per wavefront
    int nbands, nsuper;
};

// Launch shape of the EDP scans for a problem and an optional tuning.
edp_status pick_launch(const edp_problem* p, const edp_tuning* tu, Launch* L) {
    edp_status st = pick_tile(p, tu, &L->tile);
    if (st != EDP_OK) return st;
    const int g = group_of(L->tile);
    int split = (tu && tu->split > 0) ? tu->split : 1;
    if (split != 1 && split != 2) return EDP_E_INVALID;
    if (split * g > 64) return EDP_E_INVALID;
    int waves = (tu && tu->waves > 0) ? tu->waves : 4;
    if (waves > 8) return EDP_E_INVALID;
    L->split = split;
    L->waves = waves;
    // progress publication period and LDS ring depth are powers of two (masks, no division)
    int chunk = (tu && tu->chunk > 0) ? tu->chunk : 4;
    int c2 = 1;
    while (c2 < chunk && c2 < 1024) c2 <<= 1;
    L->chunk = c2;
    const int qt = qt_of(L->tile);
    int ring = 16;
    while (ring > 2 && (size_t)(waves - 1) * ring * qt * 4 > 48 * 1024) ring >>= 1;
    L->ring = ring;
    L->rpw = 64 / (split * g);
    L->nbands = (p->height + L->rpw - 1) / L->rpw;
    L->nsuper = (L->nbands + waves - 1) / waves;
    return EDP_OK;
}

struct EdpLayout {
    size_t t[4];
    size_t ctrl;        // flags, tickets, error word (uint32)
    size_t nflags, ntickets, nctrl;
    size_t total;
};

EdpLayout edp_layout(const edp_problem* p, const Launch& la) {
    EdpLayout L{};
    const size_t cells = (size_t)p->width * p->height;
    const size_t tbytes = up(cells * (size_t)qt_of(la.tile) * 4);
    size_t off = 0;
    for (int k = 0; k < 4; ++k) {
        L.t[k] = off;
        off += tbytes;
    }
    L.nflags = (size_t)la.nsuper;
    L.ntickets = (size_t)4 * p->iterations;
    L.nctrl = L.nflags + L.ntickets + 1;
    L.ctrl = off;
    off += up(L.nctrl * 4);
    L.total = off;
    return L;
}

struct DpLayout {
    size_t ptr, row_label, row_energy, total;
};

DpLayout dp_layout(const edp_problem* p, int tile) {
    DpLayout L{};
    const size_t cells = (size_t)p->width * p->height;
    const size_t pbytes = qt_of(tile) <= 256 ? 1 : 2;
    size_t off = 0;
    L.ptr = off;
    off += up(cells * (size_t)qt_of(tile) * pbytes);
    L.row_label = off;
    off += up((size_t)p->height * 4);
    L.row_energy = off;
    off += up((size_t)p->height * 8);
    L.total = off;
    return L;
}

edp_status hip_status(hipError_t e) { return e == hipSuccess ? EDP_OK : EDP_E_HIP; }

__global__ void flag_error_kernel(const uint32_t* error, int64_t* energy) {
    if (threadIdx.x == 0 && *error != 0) *energy = INT64_MIN;
}

edp_status enqueue_energy(const edp_problem* p, const void* cost, const int32_t* labels, int grid4,
                          int64_t* energy, int64_t* invalid, hipStream_t s) {
    EnergyArgs e{};
    e.cost = cost;
    e.labels = labels;
    e.energy = (unsigned long long*)energy;
    e.invalid = (unsigned long long*)invalid;
    e.W = p->width;
    e.H = p->height;
    e.qx = p->qx;
    e.qy = p->qy;
    e.lam = p->lambda;
    e.trunc = p->trunc;
    e.joint = p->trunc_mode == EDP_TRUNC_JOINT;
    e.grid4 = grid4;
    hipError_t err = launch_fill_u32((uint32_t*)energy, 2, 0, s);
    if (err == hipSuccess && invalid) err = launch_fill_u32((uint32_t*)invalid, 2, 0, s);
    if (err == hipSuccess) err = launch_energy(p->dtype, e, s);
    return hip_status(err);
}

}  // namespace

TileShape tile_shape(int tile) { return kTiles[tile]; }

}  // namespace edp

using namespace edp;

extern "C" {

edp_status edp_workspace_size(const edp_problem* prob, int32_t op, const edp_tuning* tuning, size_t* bytes) {
    if (!bytes || (op != EDP_OP_DP && op != EDP_OP_EDP)) return EDP_E_INVALID;
    edp_status st = check_problem(prob, op);
    if (st != EDP_OK) return st;
    if (op == EDP_OP_DP) {
        int tile = 0;
        st = pick_tile(prob, tuning, &tile);
        if (st != EDP_OK) return st;
        *bytes = dp_layout(prob, tile).total;
        return EDP_OK;
    }
    Launch la{};
    st = pick_launch(prob, tuning, &la);
    if (st != EDP_OK) return st;
    *bytes = edp_layout(prob, la).total;
    return EDP_OK;
}

edp_status edp_dp_scanline(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                           int32_t* d_labels, int64_t* d_row_energy, int64_t* d_energy, void* d_ws,
                           size_t ws_bytes, void* stream) {
    edp_status st = check_problem(prob, EDP_OP_DP);
    if (st != EDP_OK) return st;
    if (!d_cost || !d_labels) return EDP_E_INVALID;
    if (tuning && (tuning->chunk < 0 || tuning->n_events < 0)) return EDP_E_INVALID;
    int tile = 0;
    st = pick_tile(prob, tuning, &tile);
    if (st != EDP_OK) return st;
    // the DP kernels address the cost volume and the choice indexes with 32-bit byte offsets
    const int64_t cells = (int64_t)prob->width * prob->height;
    if (cells * qt_of(tile) * (qt_of(tile) <= 256 ? 1 : 2) >= 0x7FFF0000LL ||
        cells * prob->qx * prob->qy * (prob->dtype == EDP_I16 ? 2 : 4) >= 0x7FFF0000LL)
        return EDP_E_UNSUPPORTED;
    const DpLayout L = dp_layout(prob, tile);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < L.total) return EDP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;

    DpArgs a{};
    a.cost = d_cost;
    a.ptr = ws + L.ptr;
    a.row_label = (int32_t*)(ws + L.row_label);
    a.row_energy = (int64_t*)(ws + L.row_energy);
    a.W = prob->width;
    a.H = prob->height;
    a.qx = prob->qx;
    a.qy = prob->qy;
    a.lam = prob->lambda;
    a.clipd = prob->lambda * prob->trunc;
    a.joint = prob->trunc_mode == EDP_TRUNC_JOINT;
    a.ibits = ibits_of(prob->qx * prob->qy);
    const int rows_per_block = (64 / group_of(tile)) * 4;
    const int grid = (prob->height + rows_per_block - 1) / rows_per_block;
    // optional caller events: [0],[1] around the forward sweep, [2],[3] around the backtracking
    auto mark = [&](int k) -> bool {
        return !(tuning && tuning->events && k < tuning->n_events) ||
               hipEventRecord((hipEvent_t)tuning->events[k], s) == hipSuccess;
    };
    if (!mark(0)) return EDP_E_HIP;
    hipError_t err = launch_dp_forward(tile, prob->dtype, a, grid, s);
    if (err != hipSuccess || !mark(1)) return EDP_E_HIP;

    BtArgs b{};
    b.ptr = a.ptr;
    b.row_label = a.row_label;
    b.labels = d_labels;
    b.W = prob->width;
    b.H = prob->height;
    b.qx = prob->qx;
    b.qy = prob->qy;
    const int pbytes = qt_of(tile) <= 256 ? 1 : 2;
    b.chunk = 32768 / (qt_of(tile) * pbytes);
    if (b.chunk < 1) b.chunk = 1;
    if (!mark(2)) return EDP_E_HIP;
    err = launch_dp_backtrack(tile, b, s);
    if (err != hipSuccess || !mark(3)) return EDP_E_HIP;
    if (d_row_energy) {
        err = launch_copy_i64(a.row_energy, d_row_energy, prob->height, s);
        if (err != hipSuccess) return EDP_E_HIP;
    }
    if (d_energy) {
        err = launch_sum_rows(a.row_energy, prob->height, d_energy, s);
        if (err != hipSuccess) return EDP_E_HIP;
    }
    return EDP_OK;
}

edp_status edp_solve(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost, int32_t* d_labels,
                     int64_t* d_energy, void* d_ws, size_t ws_bytes, void* stream) {
    edp_status st = check_problem(prob, EDP_OP_EDP);
    if (st != EDP_OK) return st;
    if (!d_cost || !d_labels) return EDP_E_INVALID;
    if (tuning && (tuning->chunk < 0 || tuning->n_events < 0)) return EDP_E_INVALID;
    Launch la{};
    st = pick_launch(prob, tuning, &la);
    if (st != EDP_OK) return st;
    const int tile = la.tile;
    // the scan kernel addresses each array with 32-bit byte offsets below 0x7FFF0000
    const int64_t cells = (int64_t)prob->width * prob->height;
    if (cells * qt_of(tile) * 4 >= 0x7FFF0000LL ||
        cells * prob->qx * prob->qy * (prob->dtype == EDP_I16 ? 2 : 4) >= 0x7FFF0000LL)
        return EDP_E_UNSUPPORTED;
    const EdpLayout L = edp_layout(prob, la);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < L.total) return EDP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    uint32_t* ctrl = (uint32_t*)(ws + L.ctrl);
    uint32_t* flags = ctrl;
    uint32_t* tickets = ctrl + L.nflags;
    uint32_t* error = tickets + L.ntickets;

    hipError_t err = launch_fill_u32(ctrl, L.nctrl, 0, s);
    if (err != hipSuccess) return EDP_E_HIP;

    PassArgs a{};
    a.cost = d_cost;
    for (int k = 0; k < 4; ++k) a.t[k] = (int32_t*)(ws + L.t[k]);
    a.flags = flags;
    a.error = error;
    a.W = prob->width;
    a.H = prob->height;
    a.qx = prob->qx;
    a.qy = prob->qy;
    a.lam = prob->lambda;
    a.clipd = prob->lambda * prob->trunc;
    a.joint = prob->trunc_mode == EDP_TRUNC_JOINT;
    a.chunk = la.chunk;
    a.nbands = la.nbands;
    a.nsuper = la.nsuper;
    a.ring = la.ring;
    // cost kind of the scan kernel: int16 costs load in dword pairs when every lane's run of
    // labels starts on a 4-byte boundary
    int kind = prob->dtype == EDP_I16 ? 1 : 2;
    if (kind == 1 && kTiles[tile].kx % 2 == 0 && (prob->qx * prob->qy) % 2 == 0 &&
        (prob->qy == 1 || prob->qx % 2 == 0) && ((uintptr_t)d_cost % 4) == 0)
        kind = 3;
    const int cap = pass_capacity(tile, kind, la.split, la.waves, pass_lds_bytes(qt_of(tile), la.waves, la.ring));
    const int grid = a.nsuper < cap ? a.nsuper : cap;
    // scans P1..P4: (sx, sy) and the arrays they write (0 +x, 1 -x, 2 +y, 3 -y)
    const int sx[4] = {1, -1, 1, -1}, sy[4] = {1, 1, -1, -1};
    const int ka[4] = {0, 1, 0, 1}, kb[4] = {2, 2, 3, 3};
    int pass_index = 0;
    for (int it = 0; it < prob->iterations; ++it) {
        for (int p = 0; p < 4; ++p, ++pass_index) {
            a.sx = sx[p];
            a.sy = sy[p];
            a.ka = ka[p];
            a.kb = kb[p];
            // arrays not yet written in this solve still hold S = 0, i.e. T = M(0) = 0
            a.old_a_zero = (it == 0 && p == 0) ? 1 : 0;            // -x before P2
            a.old_b_zero = (it == 0 && (p == 0 || p == 1)) ? 1 : 0; // -y before P3
            a.ticket = tickets + pass_index;
            a.epoch = (uint32_t)pass_index * (uint32_t)(prob->width + 1);
            a.b_live = (p == 1 || p == 3) ? 1 : 0;   // T+y of P1 and T-y of P3 die inside their scan
            const bool timed = tuning && tuning->events && 2 * pass_index + 1 < tuning->n_events;
            if (timed && hipEventRecord((hipEvent_t)tuning->events[2 * pass_index], s) != hipSuccess)
                return EDP_E_HIP;
            err = launch_edp_pass(tile, kind, la.split, a, grid, la.waves, s);
            if (err != hipSuccess) return EDP_E_HIP;
            if (timed && hipEventRecord((hipEvent_t)tuning->events[2 * pass_index + 1], s) != hipSuccess)
                return EDP_E_HIP;
        }
    }
    AggArgs g{};
    g.cost = d_cost;
    for (int k = 0; k < 4; ++k) g.t[k] = a.t[k];
    g.labels = d_labels;
    g.W = prob->width;
    g.H = prob->height;
    g.qx = prob->qx;
    g.qy = prob->qy;
    const int64_t per_block = (64 / group_of(tile)) * 4;
    int64_t agrid = (cells + per_block - 1) / per_block;
    if (agrid > 8192) agrid = 8192;
    err = launch_edp_aggregate(tile, prob->dtype, g, (int)agrid, s);
    if (err != hipSuccess) return EDP_E_HIP;
    if (d_energy) {
        st = enqueue_energy(prob, d_cost, d_labels, 1, d_energy, nullptr, s);
        if (st != EDP_OK) return st;
        hipLaunchKernelGGL(flag_error_kernel, dim3(1), dim3(64), 0, s, error, d_energy);
        if (hipGetLastError() != hipSuccess) return EDP_E_HIP;
    }
    return EDP_OK;
}

edp_status edp_energy(const edp_problem* prob, const void* d_cost, const int32_t* d_labels, int32_t grid4,
                      int64_t* d_energy, int64_t* d_invalid, void* stream) {
    edp_status st = check_problem(prob, EDP_OP_DP);
    if (st == EDP_E_RANGE) st = EDP_OK;  // the energy itself is accumulated in int64
    if (st != EDP_OK) return st;
    if (!d_cost || !d_labels || !d_energy || (grid4 != 0 && grid4 != 1)) return EDP_E_INVALID;
    return enqueue_energy(prob, d_cost, d_labels, grid4, d_energy, d_invalid, (hipStream_t)stream);
}

int32_t edp_tiles(int32_t qx, int32_t qy, int32_t* ids, int32_t max) {
    if (qx < 1 || qy < 1 || max < 0) return EDP_E_INVALID;
    int n = 0;
    for (int t = 0; t < NUM_TILES; ++t) {
        if (!fits(t, qx, qy)) continue;
        if (ids && n < max) ids[n] = t;
        ++n;
    }
    return n;
}

edp_status edp_tile_info(int32_t tile, int32_t* px, int32_t* kx, int32_t* py, int32_t* ky) {
    if (tile < 0 || tile >= NUM_TILES || !px || !kx || !py || !ky) return EDP_E_INVALID;
    *px = kTiles[tile].px;
    *kx = kTiles[tile].kx;
    *py = kTiles[tile].py;
    *ky = kTiles[tile].ky;
    return EDP_OK;
}

const char* edp_status_string(int32_t status) {
    switch (status) {
        case EDP_OK: return "ok";
        case EDP_E_INVALID: return "invalid argument";
        case EDP_E_RANGE: return "int32 range guard failed";
        case EDP_E_WORKSPACE: return "workspace missing, misaligned or too small";
        case EDP_E_HIP: return "HIP runtime error";
        case EDP_E_UNSUPPORTED: return "unsupported problem";
    }
    return "unknown status";
}

}  // extern "C"
