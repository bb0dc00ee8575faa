// C ABI of the gfx950 scanline-DP / EDP library: argument checks, workspace
// layout and the order of kernel launches (Mozerov, arXiv 1410.7922,
// Algorithm 1 for edp_solve, Sec. 2 eq. base and Sec. 4.1 for the DP).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/edp.h"
#include "edp_internal.hpp"

namespace edp {

static_assert(STATUS_TIMEOUT == EDP_E_TIMEOUT, "status word value of a timed-out solve");

namespace {

// Tiles by id: single-wavefront tiles (one or two label dimensions), the wide-vertex tiles as
// 16 x (4 NV) lane grids, the single-wavefront tiles of three-dimensional label spaces, the
// wide-vertex tiles of three-dimensional label spaces (8 x 8 lanes, the third dimension over
// the NV wavefronts).
enum TileKind { TK_NONE = 0, TK_REG = 1, TK_WIDE = 2, TK_3D = 3, TK_WIDE3 = 4 };
struct TileRow {
    TileShape s;
    int kind;
    int nv;     // wavefronts per vertex
};
struct TileTable {
    TileRow t[NUM_ALL_TILES];
};
constexpr TileTable make_tiles() {
    TileTable r{};
#define EDP_ROW(id, px, kx, py, ky) r.t[id] = TileRow{{px, kx, py, ky, 1}, TK_REG, 1};
    EDP_TILE_LIST(EDP_ROW)
#undef EDP_ROW
#define EDP_MV_ROW(id, kx, ky, nv) r.t[id] = TileRow{{16, kx, 4 * nv, ky, 1}, TK_WIDE, nv};
    EDP_MV_TILE_LIST(EDP_MV_ROW)
#undef EDP_MV_ROW
#define EDP_ROW3(id, px, kx, py, ky, kz) r.t[id] = TileRow{{px, kx, py, ky, kz}, TK_3D, 1};
    EDP_TILE3_LIST(EDP_ROW3)
#undef EDP_ROW3
#define EDP_MV3_ROW(id, kz, nv) r.t[id] = TileRow{{8, 1, 8, 1, kz * nv}, TK_WIDE3, nv};
    EDP_MV3_TILE_LIST(EDP_MV3_ROW)
#undef EDP_MV3_ROW
    return r;
}
constexpr TileTable kTileTable = make_tiles();
struct TileIndex {
    const TileShape& operator[](int id) const { return kTileTable.t[id].s; }
};
constexpr TileIndex kTiles{};
int kind_of(int tile) { return tile >= 0 && tile < NUM_ALL_TILES ? kTileTable.t[tile].kind : TK_NONE; }

// tiles of the wide-vertex scan kernel (two- and three-dimensional label spaces)
bool is_wide(int tile) { return kind_of(tile) == TK_WIDE || kind_of(tile) == TK_WIDE3; }
// tiles of the single-wavefront scan kernel (two- and three-dimensional label spaces)
bool is_regular(int tile) { return kind_of(tile) == TK_REG || kind_of(tile) == TK_3D; }
int wide_nv(int tile) { return kTileTable.t[tile].nv; }

// labels along the third label dimension (0 in the problem means none)
int qz_of(const edp_problem* p) { return p->qz > 1 ? p->qz : 1; }
int64_t labels_of(const edp_problem* p) { return (int64_t)p->qx * p->qy * qz_of(p); }

constexpr size_t kAlign = 256;
size_t up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

int qt_of(int tile) {
    const TileShape& t = kTiles[tile];
    return t.px * t.py * t.kx * t.ky * t.kz;
}
int group_of(int tile) { return kTiles[tile].px * kTiles[tile].py; }
int elems_of(int tile) { return kTiles[tile].kx * kTiles[tile].ky * kTiles[tile].kz; }

bool fits(int tile, int qx, int qy, int qz = 1) {
    const TileShape& t = kTiles[tile];
    return t.px * t.kx >= qx && t.py * t.ky >= qy && t.kz >= qz;
}

// Built-in choice: least padding; then, for one label dimension, vertices that fill
// one 16-lane row (every cross-lane step of the minimum search is a single DPP
// instruction), for two, vertices that fill the wavefront (the scan step costs the
// same instructions whatever the lane count, so more lanes per vertex means fewer
// labels per lane); then fewest labels per lane; then square lane grids.
// Three label dimensions take the tiles of three-dimensional label spaces only.
int auto_tile(int qx, int qy, int qz = 1) {
    int best = -1;
    auto score = [qy, qz](int t) {
        const int lanes = group_of(t);
        const int pref = qy == 1 && qz == 1 ? 16 : 64;
        return (lanes == pref ? 0 : 1000) + 10 * elems_of(t) + (kTiles[t].px == kTiles[t].py ? 0 : 1);
    };
    for (int t = 0; t < NUM_ALL_TILES; ++t) {
        if (!is_regular(t) || (qz > 1) != (kind_of(t) == TK_3D) || !fits(t, qx, qy, qz)) continue;
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

// lambda f(T): the largest distance penalty of one label dimension, the clip of M
int64_t clip_of(const edp_problem* p) {
    const int64_t t = p->trunc;
    return (int64_t)p->lambda * (p->prior == EDP_PRIOR_SQUARED ? t * t : t);
}

// The minimum search of the scan and DP kernels for a problem (MS_*): the general RMS
// window where it has at most two steps per side (cheaper than the linear RMS then, for
// either prior), else the linear RMS (linear prior) or the walked window (squared prior).
int ms_of(const edp_problem* p) {
    const int nw = std::max({std::min(p->trunc, p->qx), std::min(p->trunc, p->qy), std::min(p->trunc, qz_of(p))}) - 1;
    if (nw <= 1) return MS_WINDOW1;
    if (nw <= 2) return MS_WINDOW;
    return p->prior == EDP_PRIOR_SQUARED ? MS_WALK : MS_LINEAR;
}

int64_t vmax_of(const edp_problem* p) {
    const int64_t dims = p->trunc_mode == EDP_TRUNC_PER_DIM ? 1 + (p->qy > 1) + (qz_of(p) > 1) : 1;
    return clip_of(p) * dims;
}

// op: an edp_op, or OP_ENERGY (the energy of a labelling: no int32 range guard applies)
constexpr int OP_ENERGY = -1;

edp_status check_problem(const edp_problem* p, int op) {
    if (!p) return EDP_E_INVALID;
    if (p->width < 1 || p->height < 1 || p->qx < 1 || p->qy < 1 || p->qz < 0) return EDP_E_INVALID;
    if ((int64_t)p->width * p->height > (int64_t)1 << 30) return EDP_E_INVALID;
    if (labels_of(p) > 4096) return EDP_E_INVALID;
    // three label dimensions: the EDP solve and the energy
    if (qz_of(p) > 1 && op != EDP_OP_EDP && op != OP_ENERGY) return EDP_E_UNSUPPORTED;
    if (p->dtype != EDP_I16 && p->dtype != EDP_I32) return EDP_E_INVALID;
    if (p->trunc_mode != EDP_TRUNC_PER_DIM && p->trunc_mode != EDP_TRUNC_JOINT) return EDP_E_INVALID;
    if (p->lambda < 0 || p->lambda > 65535 || p->trunc < 1 || p->trunc > 4096) return EDP_E_INVALID;
    if (p->prior != EDP_PRIOR_LINEAR && p->prior != EDP_PRIOR_SQUARED) return EDP_E_INVALID;
    if (p->cost_bound < 0) return EDP_E_INVALID;
    if (op == EDP_OP_EDP) {
        if (p->iterations < 1 || p->iterations > 4096) return EDP_E_INVALID;
        if ((int64_t)4 * p->iterations * ((int64_t)p->width + 1) >= ((int64_t)1 << 31)) return EDP_E_INVALID;
    }
    const int64_t b = cost_bound_of(p);
    if (b < 0) return EDP_E_INVALID;  // int32 costs need a declared bound
    // the min-marginal DP stores its forward terms, which stay within [0, Vmax], in 16 bits
    if (op == EDP_OP_DP_MARGINALS && vmax_of(p) > 65535) return EDP_E_RANGE;
    if (op == EDP_OP_EDP) {
        // empirical int32 guard for the EDP sums (they grow with the grid extent)
        if ((int64_t)(p->width + p->height) * (b + 4 * vmax_of(p)) * 8 >= ((int64_t)1 << 29)) return EDP_E_RANGE;
    } else if (op != OP_ENERGY) {
        const int64_t q = (int64_t)p->qx * p->qy;
        const int64_t span = b + vmax_of(p) + (int64_t)p->lambda * (p->qx + p->qy + 64);
        if ((span << ibits_of((int)q)) >= ((int64_t)1 << 28)) return EDP_E_RANGE;
    }
    return EDP_OK;
}

edp_status pick_tile(const edp_problem* p, const edp_tuning* tu, int* tile) {
    int t = (tu && tu->tile >= 0) ? tu->tile : auto_tile(p->qx, p->qy, qz_of(p));
    if (t < 0) return EDP_E_UNSUPPORTED;
    if (!is_regular(t) || !fits(t, p->qx, p->qy, qz_of(p))) return EDP_E_INVALID;
    *tile = t;
    return EDP_OK;
}

struct Launch {
    int tile, split, waves, chunk, ring, fuse;   // wide tiles: waves = scanlines per workgroup
    int rpw;            // scanlines per wavefront
    int nbands, nsuper;
};

// Tags of the wide tiles' hand-off words (scan, workgroup band, column) must stay distinct
// within a solve.
bool wide_tags_fit(const edp_problem* p, int64_t nsuper) {
    return (int64_t)4 * p->iterations * nsuper * ((int64_t)p->width + 1) + p->width + 2 < ((int64_t)1 << 32);
}

// Launch shape of the wide-vertex scans: scanlines per workgroup (at most 12 wavefronts) and
// LDS ring depth (largest power of two up to 8 that fits the 160 KB of LDS with the exchange
// planes).
edp_status pick_wide_launch(const edp_problem* p, const edp_tuning* tu, int tile, Launch* L) {
    const int ms = ms_of(p);
    if (ms != MS_WINDOW && ms != MS_WINDOW1) return EDP_E_UNSUPPORTED;
    if (tu && tu->split > 1) return EDP_E_INVALID;
    const int nv = wide_nv(tile);
    const int max_rows = MV_MAX_WAVES / nv;
    constexpr size_t kLds = 160 * 1024;
    // built-in: 8 compute wavefronts per workgroup (two per SIMD: a third scanline per workgroup
    // saves workgroup hand-offs but costs more in shared issue slots), as many as fit the LDS
    int rows = std::min(max_rows, std::max(1, 8 / nv));
    while (rows > 1 && pass_mv_lds_bytes(tile, ms, rows, 4) > kLds) --rows;
    if (tu && tu->waves > 0) rows = tu->waves;
    if (rows > max_rows) return EDP_E_INVALID;
    const int fuse = (tu && tu->fuse > 0) ? tu->fuse : 2;
    if (fuse != 1 && fuse != 2) return EDP_E_INVALID;
    int ring = 8;
    while (ring > 2 && pass_mv_lds_bytes(tile, ms, rows, ring) > kLds) ring >>= 1;
    if (pass_mv_lds_bytes(tile, ms, rows, ring) > kLds) return EDP_E_UNSUPPORTED;
    L->tile = tile;
    L->split = 1;
    L->waves = rows;
    L->fuse = fuse;
    L->chunk = 1;
    L->ring = ring;
    L->rpw = 1;
    L->nbands = p->height;
    L->nsuper = (p->height + rows - 1) / rows;
    if (!wide_tags_fit(p, L->nsuper)) return EDP_E_UNSUPPORTED;
    return EDP_OK;
}

// Built-in choice for the EDP scans: with two or three label dimensions and a window search, a
// wide-vertex tile unless a single-wavefront tile needs fewer padded labels (a vertex on two or
// more wavefronts shortens the dependent step: measured 2.2 against 2.7 ms for 15x15 labels at
// 320x240, 9.3 against 17 ms for 31x31 at 640x480, 8.7 against 13.1 ms for 7x7x7 at 640x480);
// among wide tiles the fewest padded labels, then the most wavefronts per vertex.  Otherwise the
// single-wavefront choice.
int auto_scan_tile(const edp_problem* p) {
    const int t = auto_tile(p->qx, p->qy, qz_of(p));
    const int ms = ms_of(p);
    const bool three = qz_of(p) > 1;
    if ((!three && p->qy < 2) || (ms != MS_WINDOW && ms != MS_WINDOW1)) return t;
    int best = -1;
    for (int w = 0; w < NUM_ALL_TILES; ++w) {
        if (kind_of(w) != (three ? TK_WIDE3 : TK_WIDE) || !fits(w, p->qx, p->qy, qz_of(p))) continue;
        if (best < 0 || qt_of(w) < qt_of(best) || (qt_of(w) == qt_of(best) && wide_nv(w) > wide_nv(best))) best = w;
    }
    if (best < 0 || (t >= 0 && qt_of(t) < qt_of(best))) return t;
    Launch la{};
    return pick_wide_launch(p, nullptr, best, &la) == EDP_OK ? best : t;
}

// Launch shape of the EDP scans for a problem and an optional tuning.
edp_status pick_launch(const edp_problem* p, const edp_tuning* tu, Launch* L) {
    const int want = (tu && tu->tile >= 0) ? tu->tile : auto_scan_tile(p);
    if (want < 0) return EDP_E_UNSUPPORTED;
    if (is_wide(want)) {
        if (!fits(want, p->qx, p->qy, qz_of(p))) return EDP_E_INVALID;
        return pick_wide_launch(p, tu, want, L);
    }
    edp_tuning t1{};
    if (tu) t1 = *tu;
    t1.tile = want;
    edp_status st = pick_tile(p, &t1, &L->tile);
    if (st != EDP_OK) return st;
    const int g = group_of(L->tile);
    int split = (tu && tu->split > 0) ? tu->split : 1;
    if (split != 1 && split != 2) return EDP_E_INVALID;
    if (split * g > 64) return EDP_E_INVALID;
    int waves = (tu && tu->waves > 0) ? tu->waves : 4;
    if (waves > MAX_WAVES) return EDP_E_INVALID;
    const int fuse = (tu && tu->fuse > 0) ? tu->fuse : 2;
    if (fuse != 1 && fuse != 2) return EDP_E_INVALID;
    L->fuse = fuse;
    L->split = split;
    L->waves = waves;
    // progress publication period and LDS ring depth are powers of two (masks, no division)
    int chunk = (tu && tu->chunk > 0) ? tu->chunk : 2;
    int c2 = 1;
    while (c2 < chunk && c2 < 1024) c2 <<= 1;
    L->chunk = c2;
    const int qt = qt_of(L->tile);
    int ring = 16;
    while (ring > 4 && (size_t)(waves + 1) * ring * qt * 4 > 96 * 1024) ring >>= 1;
    while (ring > 2 && (size_t)(waves + 1) * ring * qt * 4 > 128 * 1024) ring >>= 1;
    L->ring = ring;
    L->rpw = 64 / (split * g);
    L->nbands = (p->height + L->rpw - 1) / L->rpw;
    L->nsuper = (L->nbands + waves - 1) / waves;
    return EDP_OK;
}

// Per-instance part of an EDP workspace: the four T arrays and the flags of the
// scan launches (column progress of the first and second scan, bands done).
struct InstLayout {
    size_t t[4];
    size_t tbytes;
    size_t total;
    size_t nflags;      // uint32 words, cleared before every solve
    size_t hand_bytes;  // tagged rows between workgroup bands (cleared before every solve), or 0
};

// Tagged hand-off rows (64-bit value + tag per sum, per workgroup boundary and scan of a
// launch) are used up to this size per instance; larger instances publish column counts.
constexpr size_t kHandMax = (size_t)32 << 20;

InstLayout inst_layout(const edp_problem* p, const Launch& la) {
    InstLayout L{};
    const size_t cells = (size_t)p->width * p->height;
    L.tbytes = up(cells * (size_t)qt_of(la.tile) * 4);
    for (int k = 0; k < 4; ++k) L.t[k] = k * L.tbytes;
    L.total = 4 * L.tbytes;
    L.nflags = (size_t)3 * la.nsuper;
    const size_t hand = (size_t)2 * (la.nsuper > 1 ? la.nsuper - 1 : 0) * p->width * qt_of(la.tile) * 8;
    L.hand_bytes = la.rpw >= 2 && hand <= kHandMax ? up(hand) : 0;
    // wide tiles: two rows per scan of a launch, used by alternate workgroup bands
    if (is_wide(la.tile)) L.hand_bytes = la.nsuper > 1 ? up((size_t)4 * p->width * qt_of(la.tile) * 8) : 0;
    return L;
}

int scan_launches(const edp_problem* p, const Launch& la) { return 4 / la.fuse * p->iterations; }

// Single-instance workspace: T arrays, then the control words (flags, one
// ticket counter per scan launch, the error word) and the tagged hand-off rows,
// which every solve clears (nclear words from ctrl).
struct EdpLayout {
    InstLayout inst;
    size_t ctrl, hand;
    size_t nflags, ntickets, nctrl, nclear;
    size_t total;
};

EdpLayout edp_layout(const edp_problem* p, const Launch& la) {
    EdpLayout L{};
    L.inst = inst_layout(p, la);
    L.nflags = L.inst.nflags;
    L.ntickets = (size_t)scan_launches(p, la);
    L.nctrl = L.nflags + L.ntickets + 1;
    L.ctrl = L.inst.total;
    L.hand = L.ctrl + up(L.nctrl * 4);
    L.total = L.hand + L.inst.hand_bytes;
    L.nclear = (L.total - L.ctrl) / 4;
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

// Min-marginal DP: u16 forward terms [cells][QT], row optima [H] int64.
struct DpmLayout {
    size_t fwd, row_energy, total;
};

DpmLayout dpm_layout(const edp_problem* p, int tile) {
    DpmLayout L{};
    const size_t cells = (size_t)p->width * p->height;
    L.fwd = 0;
    L.row_energy = up(cells * (size_t)qt_of(tile) * 2);
    L.total = L.row_energy + up((size_t)p->height * 8);
    return L;
}

edp_status hip_status(hipError_t e) { return e == hipSuccess ? EDP_OK : EDP_E_HIP; }

// Batch: clear the energy words before the energy kernel adds into them.
__global__ void zero_energies_kernel(const InstDesc* descs, int32_t n) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (descs[i].energy) *descs[i].energy = 0ull;
}

// Cost kind of the scan kernel: int16 costs load in dword pairs when every
// lane's run of labels starts on a 4-byte boundary.
int cost_kind(const edp_problem* p, int tile, const void* cost) {
    int kind = p->dtype == EDP_I16 ? 1 : 2;
    if (kind == 1 && kTiles[tile].kx % 2 == 0 && labels_of(p) % 2 == 0 &&
        ((p->qy == 1 && qz_of(p) == 1) || p->qx % 2 == 0) && ((uintptr_t)cost % 4) == 0)
        kind = 3;
    return kind;
}

// The scan kernel addresses each array with 32-bit byte offsets below 0x7FFF0000.
bool edp_offsets_fit(const edp_problem* p, int tile) {
    const int64_t cells = (int64_t)p->width * p->height;
    return cells * qt_of(tile) * 4 < 0x7FFF0000LL &&
           cells * labels_of(p) * (p->dtype == EDP_I16 ? 2 : 4) < 0x7FFF0000LL;
}

InstDesc make_desc(const edp_problem* p, const Launch& la, const InstLayout& L, char* base,
                   uint32_t* flags, char* hand, const void* cost, int32_t* labels, int64_t* energy) {
    InstDesc d{};
    d.cost = cost;
    d.hand = L.hand_bytes ? (unsigned long long*)hand : nullptr;
    for (int k = 0; k < 4; ++k) d.t[k] = (int32_t*)(base + L.t[k]);
    d.labels = labels;
    d.energy = (unsigned long long*)energy;
    d.flags = flags;
    d.W = p->width;
    d.H = p->height;
    d.qx = p->qx;
    d.qy = p->qy;
    d.qz = qz_of(p);
    d.lam = p->lambda;
    d.clipd = (int32_t)clip_of(p);
    d.joint = p->trunc_mode == EDP_TRUNC_JOINT;
    d.trunc = p->trunc;
    d.squared = p->prior == EDP_PRIOR_SQUARED;
    d.nbands = la.nbands;
    d.nsuper = la.nsuper;
    return d;
}

// Everything one launch shape needs to run its scans and the marginal.
struct ClassRun {
    int tile, kind, dtype, split, waves, chunk, ring, fuse, iterations;
    int ms;                    // minimum search kind MS_*
    InstDesc one;              // single instance (descs null)
    const InstDesc* descs;     // device descriptor slice of a batch class
    int ndesc;
    int tickets_per_pass;
    int agg_blocks, cells_per_block;
    uint32_t* tickets;         // one counter per scan launch
    uint32_t* error;
    int64_t sums_bytes;        // bytes of one array of sums over the class's instances
};

// Memory-side cache (Infinity Cache) of the device: where one array of sums is larger, a later scan
// finds none of it there, and the wide-tile scans stream the sums with non-temporal accesses.
constexpr int64_t kMallBytes = (int64_t)256 << 20;

int64_t sums_bytes_of(const edp_problem& p, int tile) { return (int64_t)p.width * p.height * qt_of(tile) * 4; }

int agg_cells_per_block(int tile) { return is_wide(tile) ? 4 : (64 / group_of(tile)) * 4; }

int scan_grid(const ClassRun& c) {
    const int cap =
        is_wide(c.tile)
            ? pass_mv_capacity(c.tile, c.kind, c.ms, c.waves, pass_mv_lds_bytes(c.tile, c.ms, c.waves, c.ring))
            : pass_capacity(c.tile, c.kind, c.split, c.ms, c.waves, pass_lds_bytes(qt_of(c.tile), c.waves, c.ring));
    const int total = c.fuse * c.tickets_per_pass;
    return total < cap ? total : cap;
}

// Scans P1..P4 of Algorithm 1 (arrays 0 +x, 1 -x, 2 +y, 3 -y), iterations
// times, then the marginal of eq. DP_2D_1 with its smallest argmin.
edp_status enqueue_class(const ClassRun& c, const edp_tuning* ev, hipStream_t s) {
    static const int sx[4] = {1, -1, 1, -1}, sy[4] = {1, 1, -1, -1};
    static const int ka[4] = {0, 1, 0, 1}, kb[4] = {2, 2, 3, 3};
    PassArgs a{};
    a.one = c.one;
    a.descs = c.descs;
    a.ndesc = c.descs ? c.ndesc : 0;
    a.tickets_per_pass = c.tickets_per_pass;
    a.npass = c.fuse;
    a.error = c.error;
    a.chunk = c.chunk;
    a.ring = c.ring;
    const int grid = scan_grid(c);
    int launch = 0;
    for (int it = 0; it < c.iterations; ++it) {
        for (int p = 0; p < 4; p += c.fuse, ++launch) {
            for (int k = 0; k < c.fuse; ++k) {
                const int q = p + k;
                PassDir& d = a.dir[k];
                d.sx = sx[q];
                d.sy = sy[q];
                d.ka = ka[q];
                d.kb = kb[q];
                // arrays not yet written in this solve still hold S = 0, i.e. T = M(0) = 0
                d.old_a_zero = (it == 0 && q == 0) ? 1 : 0;             // -x before P2
                d.old_b_zero = (it == 0 && (q == 0 || q == 1)) ? 1 : 0;  // -y before P3
                d.b_live = (q == 1 || q == 3) ? 1 : 0;  // T+y of P1 and T-y of P3 die inside their scan
                d.pass_index = it * 4 + q;
                d.marginal = (is_wide(c.tile) && q == 3 && it == c.iterations - 1) ? 1 : 0;
            }
            a.ticket = c.tickets + launch;
            const bool timed = ev && ev->events && 2 * launch + 1 < ev->n_events;
            if (timed && hipEventRecord((hipEvent_t)ev->events[2 * launch], s) != hipSuccess) return EDP_E_HIP;
            const hipError_t le = is_wide(c.tile) ? launch_edp_pass_mv(c.tile, c.kind, c.ms, a, grid, c.waves, s,
                                                                       c.sums_bytes > kMallBytes)
                                                  : launch_edp_pass(c.tile, c.kind, c.split, c.ms, a, grid, c.waves, s);
            if (le != hipSuccess) return EDP_E_HIP;
            if (timed && hipEventRecord((hipEvent_t)ev->events[2 * launch + 1], s) != hipSuccess)
                return EDP_E_HIP;
        }
    }
    if (is_wide(c.tile) && c.kind != KIND_WINDOW) {
        // a batch class writes its status words in its energy launch
        if (c.descs) return EDP_OK;
        return launch_status(c.one, nullptr, 0, c.error, s) == hipSuccess ? EDP_OK : EDP_E_HIP;
    }
    AggArgs g{};
    g.one = c.one;
    g.descs = c.descs;
    g.ndesc = a.ndesc;
    g.cells_per_block = c.cells_per_block;
    g.error = c.error;
    const hipError_t e = c.kind == KIND_WINDOW ? launch_edp_aggregate_win(g, c.agg_blocks, s)
                         : is_wide(c.tile)     ? launch_edp_aggregate_mv(c.tile, c.dtype, g, c.agg_blocks, s)
                                               : launch_edp_aggregate(c.tile, c.dtype, g, c.agg_blocks, s);
    return e == hipSuccess ? EDP_OK : EDP_E_HIP;
}

// ---------------------------------------------------------------------------
// Label-window solve
// ---------------------------------------------------------------------------

// Costs outside a window inside the 8 x 8 frames: larger than any sum the range guard allows
// for the window labels, small enough that sums with it stay inside int32.
constexpr int32_t kWinBig = 1 << 29;

// The frame problem the scans run on: 8 x 8 labels per vertex, int32 costs.
edp_problem frame_problem(const edp_problem* p) {
    edp_problem f = *p;
    f.qx = WIN_FRAME;
    f.qy = WIN_FRAME;
    f.dtype = EDP_I32;
    return f;
}

struct WinLayout {
    EdpLayout edp;       // T arrays and control words of the frame problem
    size_t cw, shifts;   // frame costs [cells][64] int32, shifts [cells][2] uint32
    size_t total;
};

edp_status win_launch(const edp_problem* prob, int32_t win, const edp_tuning* tu, Launch* la) {
    edp_status st = check_problem(prob, EDP_OP_EDP);
    if (st != EDP_OK) return st;
    if (win < 1 || win > WIN_FRAME || !(win & 1) || win > prob->qx || win > prob->qy) return EDP_E_INVALID;
    if (qz_of(prob) > 1) return EDP_E_UNSUPPORTED;   // windows of two-dimensional label spaces
    // neighbouring centres differ by at most q - win labels per axis; the frame shifts are int8
    if (prob->qx - win > 127 || prob->qy - win > 127) return EDP_E_UNSUPPORTED;
    if (prob->dtype != EDP_I32 || prob->prior != EDP_PRIOR_LINEAR) return EDP_E_UNSUPPORTED;
    if (tu && ((tu->tile >= 0 && tu->tile != WIN_TILE) || (tu->split > 1) || tu->chunk < 0 || tu->n_events < 0))
        return EDP_E_INVALID;
    edp_tuning t{};
    if (tu) t = *tu;
    t.tile = WIN_TILE;
    t.split = 1;
    const edp_problem f = frame_problem(prob);
    st = pick_launch(&f, &t, la);
    if (st != EDP_OK) return st;
    const int64_t cells = (int64_t)prob->width * prob->height;
    if (!edp_offsets_fit(&f, WIN_TILE) || cells * 8 >= 0x7FFF0000LL) return EDP_E_UNSUPPORTED;
    return EDP_OK;
}

WinLayout win_layout(const edp_problem* prob, const Launch& la) {
    WinLayout L{};
    const edp_problem f = frame_problem(prob);
    L.edp = edp_layout(&f, la);
    const size_t cells = (size_t)prob->width * prob->height;
    L.cw = L.edp.total;
    L.shifts = L.cw + up(cells * WIN_FRAME * WIN_FRAME * 4);
    L.total = L.shifts + up(cells * 8);
    return L;
}

// error (nullable): the solve's error word; zeroed: the energy word was cleared with the solve's
// control words
edp_status enqueue_energy(const edp_problem* p, const void* cost, const int32_t* labels, int grid4,
                          int64_t* energy, int64_t* invalid, hipStream_t s, const uint32_t* error = nullptr,
                          bool zeroed = false) {
    EnergyArgs e{};
    e.cost = cost;
    e.labels = labels;
    e.energy = (unsigned long long*)energy;
    e.invalid = (unsigned long long*)invalid;
    e.W = p->width;
    e.H = p->height;
    e.qx = p->qx;
    e.qy = p->qy;
    e.qz = qz_of(p);
    e.lam = p->lambda;
    e.trunc = p->trunc;
    e.joint = p->trunc_mode == EDP_TRUNC_JOINT;
    e.grid4 = grid4;
    e.squared = p->prior == EDP_PRIOR_SQUARED;
    e.error = error;
    hipError_t err = zeroed ? hipSuccess : launch_fill_u32((uint32_t*)energy, 2, 0, s);
    if (err == hipSuccess && invalid) err = launch_fill_u32((uint32_t*)invalid, 2, 0, s);
    if (err == hipSuccess) err = launch_energy(p->dtype, e, s);
    return hip_status(err);
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

constexpr int kEnergyRows = 2;   // rows per block of the batched energy kernel

struct BatchEntry {
    Launch la;
    int kind;
    InstLayout L;
    size_t base;         // byte offset of the instance's T arrays in the workspace
    size_t flags_word;   // first control word of the instance's flags
    size_t hand;         // byte offset of the instance's tagged hand-off rows
    int64_t est;         // critical-path estimate in scan steps (sort key)
};

struct BatchClassPlan {
    int tile, kind, dtype, split, waves, chunk, ring, fuse, iterations;
    int ms;
    std::vector<int> members;   // items, longest first
    int first_desc;
    size_t tickets_word, error_word;
    int tickets_per_pass, agg_blocks, cells_per_block, energy_blocks;
    int64_t sums_bytes;
};

struct BatchLayout {
    std::vector<BatchEntry> e;
    std::vector<BatchClassPlan> classes;
    size_t desc_off, ctrl_off, nctrl, total;
};

edp_status plan_batch(int32_t n, const edp_batch_item* items, BatchLayout* B) {
    if (n < 1 || n > 65536 || !items) return EDP_E_INVALID;
    B->e.assign(n, BatchEntry{});
    B->classes.clear();
    for (int i = 0; i < n; ++i) {
        const edp_batch_item& it = items[i];
        edp_status st = check_problem(&it.problem, EDP_OP_EDP);
        if (st != EDP_OK) return st;
        if (!it.d_cost || !it.d_labels) return EDP_E_INVALID;
        if (it.tuning.chunk < 0) return EDP_E_INVALID;
        BatchEntry& e = B->e[i];
        st = pick_launch(&it.problem, &it.tuning, &e.la);
        if (st != EDP_OK) return st;
        if (!edp_offsets_fit(&it.problem, e.la.tile)) return EDP_E_UNSUPPORTED;
        e.kind = cost_kind(&it.problem, e.la.tile, it.d_cost);
        e.L = inst_layout(&it.problem, e.la);
        e.est = (int64_t)it.problem.width + 4 * (int64_t)it.problem.height;
        int c = 0;
        for (; c < (int)B->classes.size(); ++c) {
            const BatchClassPlan& k = B->classes[c];
            if (k.tile == e.la.tile && k.kind == e.kind && k.split == e.la.split && k.waves == e.la.waves &&
                k.chunk == e.la.chunk && k.ring == e.la.ring && k.fuse == e.la.fuse &&
                k.iterations == it.problem.iterations && k.ms == ms_of(&it.problem))
                break;
        }
        if (c == (int)B->classes.size()) {
            BatchClassPlan k{};
            k.tile = e.la.tile;
            k.kind = e.kind;
            k.dtype = it.problem.dtype;
            k.split = e.la.split;
            k.waves = e.la.waves;
            k.chunk = e.la.chunk;
            k.ring = e.la.ring;
            k.fuse = e.la.fuse;
            k.ms = ms_of(&it.problem);
            k.iterations = it.problem.iterations;
            B->classes.push_back(k);
        }
        B->classes[c].members.push_back(i);
    }
    // workspace: descriptor table, every instance's T arrays, then the control words
    size_t off = 0;
    B->desc_off = off;
    off += up((size_t)n * sizeof(InstDesc));
    for (int i = 0; i < n; ++i) {
        B->e[i].base = off;
        off += B->e[i].L.total;
    }
    size_t word = 0;
    for (int i = 0; i < n; ++i) {
        B->e[i].flags_word = word;
        word += B->e[i].L.nflags;
    }
    int first_desc = 0;
    for (BatchClassPlan& k : B->classes) {
        std::stable_sort(k.members.begin(), k.members.end(),
                         [&](int a, int b) { return B->e[a].est > B->e[b].est; });
        k.first_desc = first_desc;
        first_desc += (int)k.members.size();
        k.cells_per_block = agg_cells_per_block(k.tile);
        int64_t tickets = 0, blocks = 0, eblocks = 0;
        k.sums_bytes = 0;
        for (int i : k.members) {
            const edp_problem& p = items[i].problem;
            k.sums_bytes += sums_bytes_of(p, k.tile);
            tickets += B->e[i].la.nsuper;
            blocks += ((int64_t)p.width * p.height + k.cells_per_block - 1) / k.cells_per_block;
            eblocks += (p.height + kEnergyRows - 1) / kEnergyRows;
        }
        if (tickets * k.fuse >= INT_MAX || blocks >= INT_MAX || eblocks >= INT_MAX) return EDP_E_UNSUPPORTED;
        k.tickets_per_pass = (int)tickets;
        k.agg_blocks = (int)blocks;
        k.energy_blocks = (int)eblocks;
        k.tickets_word = word;
        word += (size_t)4 / k.fuse * k.iterations;
        k.error_word = word;
        word += 1;
    }
    B->ctrl_off = off;
    off += up(word * 4);
    for (int i = 0; i < n; ++i) {
        B->e[i].hand = off;
        off += B->e[i].L.hand_bytes;
    }
    B->nctrl = (off - B->ctrl_off) / 4;        // control words and tagged rows, cleared each solve
    B->total = off;
    return EDP_OK;
}

}  // namespace

TileShape tile_shape(int tile) { return kTiles[tile]; }

}  // namespace edp

using namespace edp;

struct edp_batch_plan {
    int32_t n;
    char* ws;
    size_t ctrl_off, nctrl;
    const InstDesc* descs;              // device descriptor table (in the workspace)
    std::vector<BatchClassPlan> classes;
    std::vector<hipStream_t> streams;   // one per class when there are several
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
};

namespace {

void release_plan(edp_batch_plan* p) {
    for (hipStream_t st : p->streams) hipStreamDestroy(st);
    for (hipEvent_t ev : p->joins) hipEventDestroy(ev);
    if (p->fork) hipEventDestroy(p->fork);
    delete p;
}

}  // namespace

extern "C" {

edp_status edp_workspace_size(const edp_problem* prob, int32_t op, const edp_tuning* tuning, size_t* bytes) {
    if (!bytes || (op != EDP_OP_DP && op != EDP_OP_EDP && op != EDP_OP_DP_MARGINALS)) return EDP_E_INVALID;
    edp_status st = check_problem(prob, op);
    if (st != EDP_OK) return st;
    if (op == EDP_OP_DP || op == EDP_OP_DP_MARGINALS) {
        int tile = 0;
        st = pick_tile(prob, tuning, &tile);
        if (st != EDP_OK) return st;
        *bytes = op == EDP_OP_DP ? dp_layout(prob, tile).total : dpm_layout(prob, tile).total;
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
    a.clipd = (int32_t)clip_of(prob);
    a.joint = prob->trunc_mode == EDP_TRUNC_JOINT;
    a.trunc = prob->trunc;
    a.ms = ms_of(prob);
    a.squared = prob->prior == EDP_PRIOR_SQUARED;
    a.ibits = ibits_of(prob->qx * prob->qy);
    const int rows_per_block = (64 / group_of(tile)) * 4;
    const int grid = (prob->height + rows_per_block - 1) / rows_per_block;
    // optional caller events: [0],[1] around the forward sweep, [2],[3] around the backtracking
    auto mark = [&](int k) -> bool {
        return !(tuning && tuning->events && k < tuning->n_events) ||
               hipEventRecord((hipEvent_t)tuning->events[k], s) == hipSuccess;
    };
    if (!mark(0)) return EDP_E_HIP;
    hipError_t err = launch_dp_forward(tile, cost_kind(prob, tile, d_cost), a, grid, s);
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
    // columns per LDS chunk of the backtracking (16 scanlines per workgroup, about 32 KB)
    b.chunk = 32768 / (16 * qt_of(tile) * pbytes);
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
                     int64_t* d_energy, int32_t* d_status, void* d_ws, size_t ws_bytes, void* stream) {
    edp_status st = check_problem(prob, EDP_OP_EDP);
    if (st != EDP_OK) return st;
    if (!d_cost || !d_labels) return EDP_E_INVALID;
    if (tuning && (tuning->chunk < 0 || tuning->n_events < 0)) return EDP_E_INVALID;
    Launch la{};
    st = pick_launch(prob, tuning, &la);
    if (st != EDP_OK) return st;
    if (!edp_offsets_fit(prob, la.tile)) return EDP_E_UNSUPPORTED;
    const EdpLayout L = edp_layout(prob, la);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < L.total) return EDP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    uint32_t* ctrl = (uint32_t*)(ws + L.ctrl);
    uint32_t* flags = ctrl;
    uint32_t* tickets = ctrl + L.nflags;
    uint32_t* error = tickets + L.ntickets;

    // control words, and the energy word the energy kernel adds into, cleared in one launch
    if (launch_fill_u32_with(ctrl, L.nclear, (uint32_t*)d_energy, d_energy ? 2 : 0, 0, s) != hipSuccess)
        return EDP_E_HIP;
    ClassRun c{};
    c.tile = la.tile;
    c.kind = cost_kind(prob, la.tile, d_cost);
    c.dtype = prob->dtype;
    c.split = la.split;
    c.waves = la.waves;
    c.chunk = la.chunk;
    c.ring = la.ring;
    c.fuse = la.fuse;
    c.iterations = prob->iterations;
    c.ms = ms_of(prob);
    c.one = make_desc(prob, la, L.inst, ws, flags, ws + L.hand, d_cost, d_labels, nullptr);
    c.one.status = d_status;
    c.sums_bytes = sums_bytes_of(*prob, la.tile);
    c.descs = nullptr;
    c.ndesc = 1;
    c.tickets_per_pass = la.nsuper;
    c.cells_per_block = agg_cells_per_block(la.tile);
    const int64_t cells = (int64_t)prob->width * prob->height;
    c.agg_blocks = (int)((cells + c.cells_per_block - 1) / c.cells_per_block);
    c.tickets = tickets;
    c.error = error;
    st = enqueue_class(c, tuning, s);
    if (st != EDP_OK) return st;
    if (d_energy) {
        st = enqueue_energy(prob, d_cost, d_labels, 1, d_energy, nullptr, s, error, true);
        if (st != EDP_OK) return st;
    }
    return EDP_OK;
}

edp_status edp_batch_workspace_size(int32_t n, const edp_batch_item* items, size_t* bytes) {
    if (!bytes) return EDP_E_INVALID;
    BatchLayout B;
    edp_status st = plan_batch(n, items, &B);
    if (st != EDP_OK) return st;
    *bytes = B.total;
    return EDP_OK;
}

edp_status edp_batch_plan_create(int32_t n, const edp_batch_item* items, void* d_ws, size_t ws_bytes,
                                 void* stream, edp_batch_plan** plan) {
    if (!plan) return EDP_E_INVALID;
    BatchLayout B;
    edp_status st = plan_batch(n, items, &B);
    if (st != EDP_OK) return st;
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < B.total) return EDP_E_WORKSPACE;
    char* ws = (char*)d_ws;
    uint32_t* ctrl = (uint32_t*)(ws + B.ctrl_off);
    std::vector<InstDesc> descs(n);
    for (const BatchClassPlan& k : B.classes) {
        int ticket = 0, block = 0, eblock = 0;
        for (size_t m = 0; m < k.members.size(); ++m) {
            const int i = k.members[m];
            const edp_batch_item& it = items[i];
            const BatchEntry& e = B.e[i];
            InstDesc d = make_desc(&it.problem, e.la, e.L, ws + e.base, ctrl + e.flags_word, ws + e.hand,
                                   it.d_cost, it.d_labels, it.d_energy);
            d.status = it.d_status;
            d.first_ticket = ticket;
            d.first_block = block;
            d.first_eblock = eblock;
            ticket += e.la.nsuper;
            block += (int)(((int64_t)it.problem.width * it.problem.height + k.cells_per_block - 1) /
                           k.cells_per_block);
            eblock += (it.problem.height + kEnergyRows - 1) / kEnergyRows;
            descs[k.first_desc + m] = d;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(ws + B.desc_off, descs.data(), (size_t)n * sizeof(InstDesc), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return EDP_E_HIP;
    edp_batch_plan* p = new edp_batch_plan();
    p->n = n;
    p->ws = ws;
    p->ctrl_off = B.ctrl_off;
    p->nctrl = B.nctrl;
    p->descs = (const InstDesc*)(ws + B.desc_off);
    p->classes = B.classes;
    if (p->classes.size() > 1) {
        bool ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
        for (size_t c = 0; ok && c < p->classes.size(); ++c) {
            hipStream_t cs = nullptr;
            hipEvent_t ev = nullptr;
            ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
            if (ok) p->streams.push_back(cs);
            ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
            if (ok) p->joins.push_back(ev);
        }
        if (!ok) {
            release_plan(p);
            return EDP_E_HIP;
        }
    }
    *plan = p;
    return EDP_OK;
}

edp_status edp_batch_solve(const edp_batch_plan* plan, void* stream) {
    if (!plan) return EDP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* ctrl = (uint32_t*)(plan->ws + plan->ctrl_off);
    if (launch_fill_u32(ctrl, plan->nctrl, 0, s) != hipSuccess) return EDP_E_HIP;
    hipLaunchKernelGGL(zero_energies_kernel, dim3((plan->n + 255) / 256), dim3(256), 0, s, plan->descs, plan->n);
    if (hipGetLastError() != hipSuccess) return EDP_E_HIP;
    const bool fork = plan->classes.size() > 1;
    if (fork && hipEventRecord(plan->fork, s) != hipSuccess) return EDP_E_HIP;
    for (size_t ci = 0; ci < plan->classes.size(); ++ci) {
        const BatchClassPlan& k = plan->classes[ci];
        hipStream_t cs = fork ? plan->streams[ci] : s;
        if (fork && hipStreamWaitEvent(cs, plan->fork, 0) != hipSuccess) return EDP_E_HIP;
        ClassRun c{};
        c.tile = k.tile;
        c.kind = k.kind;
        c.dtype = k.dtype;
        c.split = k.split;
        c.waves = k.waves;
        c.chunk = k.chunk;
        c.ring = k.ring;
        c.fuse = k.fuse;
        c.iterations = k.iterations;
        c.ms = k.ms;
        c.descs = plan->descs + k.first_desc;
        c.ndesc = (int)k.members.size();
        c.tickets_per_pass = k.tickets_per_pass;
        c.agg_blocks = k.agg_blocks;
        c.cells_per_block = k.cells_per_block;
        c.tickets = ctrl + k.tickets_word;
        c.error = ctrl + k.error_word;
        c.sums_bytes = k.sums_bytes;
        edp_status st = enqueue_class(c, nullptr, cs);
        if (st != EDP_OK) return st;
        BatchEnergyArgs ea{};
        ea.descs = c.descs;
        ea.ndesc = c.ndesc;
        ea.rows_per_block = kEnergyRows;
        ea.error = c.error;
        ea.status = is_wide(k.tile) ? 1 : 0;   // the marginal kernel writes them for the other tiles
        if (launch_batch_energy(k.dtype, ea, k.energy_blocks, cs) != hipSuccess) return EDP_E_HIP;
        if (fork && (hipEventRecord(plan->joins[ci], cs) != hipSuccess ||
                     hipStreamWaitEvent(s, plan->joins[ci], 0) != hipSuccess))
            return EDP_E_HIP;
    }
    return EDP_OK;
}

edp_status edp_batch_plan_info(const edp_batch_plan* plan, int32_t* n_classes, int32_t* n_launches) {
    if (!plan) return EDP_E_INVALID;
    if (n_classes) *n_classes = (int32_t)plan->classes.size();
    if (n_launches) {
        int32_t l = 2;   // clear the control words and the energies
        // per class: the scan launches, the marginal (single-wavefront tiles; the wide tiles' last
        // scan forms the labels), the energies with the status words
        for (const BatchClassPlan& k : plan->classes) l += 4 / k.fuse * k.iterations + (is_wide(k.tile) ? 1 : 2);
        *n_launches = l;
    }
    return EDP_OK;
}

void edp_batch_plan_destroy(edp_batch_plan* plan) {
    if (plan) release_plan(plan);
}

edp_status edp_window_workspace_size(const edp_problem* prob, int32_t win, const edp_tuning* tuning,
                                     size_t* bytes) {
    if (!bytes) return EDP_E_INVALID;
    Launch la{};
    edp_status st = win_launch(prob, win, tuning, &la);
    if (st != EDP_OK) return st;
    *bytes = win_layout(prob, la).total;
    return EDP_OK;
}

edp_status edp_solve_windowed(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                              const int32_t* d_centers, int32_t win, int32_t* d_labels, int64_t* d_energy,
                              int32_t* d_status, void* d_ws, size_t ws_bytes, void* stream) {
    Launch la{};
    edp_status st = win_launch(prob, win, tuning, &la);
    if (st != EDP_OK) return st;
    if (!d_cost || !d_centers || !d_labels) return EDP_E_INVALID;
    const WinLayout L = win_layout(prob, la);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < L.total) return EDP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    const EdpLayout& E = L.edp;
    uint32_t* ctrl = (uint32_t*)(ws + E.ctrl);
    uint32_t* flags = ctrl;
    uint32_t* tickets = ctrl + E.nflags;
    uint32_t* error = tickets + E.ntickets;
    int32_t* cw = (int32_t*)(ws + L.cw);
    uint32_t* shifts = (uint32_t*)(ws + L.shifts);

    if (launch_fill_u32(ctrl, E.nclear, 0, s) != hipSuccess) return EDP_E_HIP;
    if (launch_win_prep((const int32_t*)d_cost, d_centers, prob->width, prob->height, prob->qx, prob->qy, win, kWinBig,
                        cw, shifts, s) != hipSuccess)
        return EDP_E_HIP;
    const edp_problem f = frame_problem(prob);
    ClassRun c{};
    c.tile = WIN_TILE;
    c.kind = KIND_WINDOW;
    c.dtype = EDP_I32;
    c.split = 1;
    c.waves = la.waves;
    c.chunk = la.chunk;
    c.ring = la.ring;
    c.fuse = la.fuse;
    c.iterations = prob->iterations;
    // the window kernel's own search between shifted frames: the general RMS window for T <= 3
    c.ms = prob->trunc <= 3 ? MS_WINDOW : MS_LINEAR;
    c.one = make_desc(&f, la, E.inst, ws, flags, ws + E.hand, cw, d_labels, nullptr);
    c.one.aux = shifts;
    c.one.centers = d_centers;
    c.one.win = win;
    c.one.qx_full = prob->qx;
    c.one.status = d_status;
    c.descs = nullptr;
    c.ndesc = 1;
    c.tickets_per_pass = la.nsuper;
    c.cells_per_block = agg_cells_per_block(WIN_TILE);
    const int64_t cells = (int64_t)prob->width * prob->height;
    c.agg_blocks = (int)((cells + c.cells_per_block - 1) / c.cells_per_block);
    c.tickets = tickets;
    c.error = error;
    st = enqueue_class(c, tuning, s);
    if (st != EDP_OK) return st;
    if (d_energy) {
        st = enqueue_energy(prob, d_cost, d_labels, 1, d_energy, nullptr, s, error);
        if (st != EDP_OK) return st;
    }
    return EDP_OK;
}

edp_status edp_dp_marginals(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                            int32_t* d_labels, int32_t* d_marginal, int64_t* d_row_energy, int64_t* d_energy,
                            void* d_ws, size_t ws_bytes, void* stream) {
    edp_status st = check_problem(prob, EDP_OP_DP_MARGINALS);
    if (st != EDP_OK) return st;
    if (!d_cost || !d_labels) return EDP_E_INVALID;
    if (tuning && (tuning->chunk < 0 || tuning->n_events < 0)) return EDP_E_INVALID;
    int tile = 0;
    st = pick_tile(prob, tuning, &tile);
    if (st != EDP_OK) return st;
    // 32-bit byte offsets: cost volume, forward terms, marginal output
    const int64_t cells = (int64_t)prob->width * prob->height;
    const int64_t q = (int64_t)prob->qx * prob->qy;
    if (cells * qt_of(tile) * 2 >= 0x7FFF0000LL || cells * q * (prob->dtype == EDP_I16 ? 2 : 4) >= 0x7FFF0000LL ||
        (d_marginal && cells * q * 4 >= 0x7FFF0000LL))
        return EDP_E_UNSUPPORTED;
    const DpmLayout L = dpm_layout(prob, tile);
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0 || ws_bytes < L.total) return EDP_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    DpmArgs a{};
    a.cost = d_cost;
    a.fwd = ws + L.fwd;
    a.labels = d_labels;
    a.marginal = d_marginal;
    a.row_energy = (int64_t*)(ws + L.row_energy);
    a.W = prob->width;
    a.H = prob->height;
    a.qx = prob->qx;
    a.qy = prob->qy;
    a.lam = prob->lambda;
    a.clipd = (int32_t)clip_of(prob);
    a.joint = prob->trunc_mode == EDP_TRUNC_JOINT;
    a.trunc = prob->trunc;
    a.ms = ms_of(prob);
    a.squared = prob->prior == EDP_PRIOR_SQUARED;
    // the DP range guard keeps (cost bound + Vmax) << ibits below 2^28, so the argmin keys
    // ((S_Omega + bias) << ibits) | label, S_Omega + bias <= 2 (cost bound + Vmax), fit
    a.bias = (int32_t)cost_bound_of(prob);
    a.ibits = ibits_of(prob->qx * prob->qy);
    const int rows_per_block = (64 / group_of(tile)) * 4;
    const int grid = (prob->height + rows_per_block - 1) / rows_per_block;
    // optional caller events: [0],[1] around the forward sweep, [2],[3] around the backward sweep
    auto mark = [&](int k) -> bool {
        return !(tuning && tuning->events && k < tuning->n_events) ||
               hipEventRecord((hipEvent_t)tuning->events[k], s) == hipSuccess;
    };
    if (!mark(0)) return EDP_E_HIP;
    hipError_t err = launch_dp_marginals(tile, prob->dtype, a, grid, true, s);
    if (err != hipSuccess || !mark(1) || !mark(2)) return EDP_E_HIP;
    err = launch_dp_marginals(tile, prob->dtype, a, grid, false, s);
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

edp_status edp_dsi(const uint8_t* d_i0, const uint8_t* d_i1, const uint8_t* d_i2, int32_t width, int32_t height,
                   int32_t qx, int32_t qy, int32_t ox, int32_t oy, int32_t sx, int32_t sy, int32_t l2, int32_t cmax,
                   int32_t dtype, void* d_cost, void* stream) {
    if (!d_i0 || !d_i1 || !d_cost) return EDP_E_INVALID;
    if (width < 1 || height < 1 || qx < 1 || qy < 1 || (int64_t)qx * qy > 4096) return EDP_E_INVALID;
    if ((int64_t)width * height > (int64_t)1 << 30) return EDP_E_INVALID;
    if ((sx != 1 && sx != -1) || (sy != 1 && sy != -1) || (l2 != 1 && l2 != 2)) return EDP_E_INVALID;
    // displacements are kept as 16-bit halves: |ox|, |oy| <= 16384 with at most 4096 labels
    if (ox < -16384 || ox > 16384 || oy < -16384 || oy > 16384) return EDP_E_INVALID;
    if (dtype != EDP_I16 && dtype != EDP_I32) return EDP_E_INVALID;
    if (cmax < 0 || (dtype == EDP_I16 && cmax > 32767)) return EDP_E_INVALID;
    const size_t esize = dtype == EDP_I16 ? 2 : 4;
    if ((uintptr_t)d_cost % esize != 0) return EDP_E_INVALID;
    DsiArgs a{};
    a.i0 = d_i0;
    a.i1 = d_i1;
    a.i2 = d_i2;
    a.cost = d_cost;
    a.W = width;
    a.H = height;
    a.qx = qx;
    a.qy = qy;
    a.ox = ox;
    a.oy = oy;
    a.sx = sx;
    a.sy = sy;
    a.l2 = l2;
    // 255^2 fits every int32 cmax; the truncation bounds the values by the output type
    a.cmax = cmax;
    a.vec = ((uintptr_t)d_cost % 16) == 0;
    a.inv_q = 1.0 / ((double)qx * qy);
    a.inv_w = 1.0 / (double)width;
    return hip_status(launch_dsi(a, dtype, (hipStream_t)stream));
}

edp_status edp_energy(const edp_problem* prob, const void* d_cost, const int32_t* d_labels, int32_t grid4,
                      int64_t* d_energy, int64_t* d_invalid, void* stream) {
    edp_status st = check_problem(prob, OP_ENERGY);   // the energy itself is accumulated in int64
    if (st != EDP_OK) return st;
    if (!d_cost || !d_labels || !d_energy || (grid4 != 0 && grid4 != 1)) return EDP_E_INVALID;
    return enqueue_energy(prob, d_cost, d_labels, grid4, d_energy, d_invalid, (hipStream_t)stream);
}

int32_t edp_tiles(int32_t qx, int32_t qy, int32_t* ids, int32_t max) {
    if (qx < 1 || qy < 1 || max < 0) return EDP_E_INVALID;
    int n = 0;
    for (int t = 0; t < NUM_ALL_TILES; ++t) {
        if (kind_of(t) != TK_REG || !fits(t, qx, qy)) continue;
        if (ids && n < max) ids[n] = t;
        ++n;
    }
    return n;
}

int32_t edp_wide_tiles(int32_t qx, int32_t qy, int32_t* ids, int32_t max) {
    if (qx < 1 || qy < 1 || max < 0) return EDP_E_INVALID;
    int n = 0;
    for (int t = 0; t < NUM_ALL_TILES; ++t) {
        if (kind_of(t) != TK_WIDE || !fits(t, qx, qy)) continue;
        if (ids && n < max) ids[n] = t;
        ++n;
    }
    return n;
}

int32_t edp_tiles_3d(int32_t qx, int32_t qy, int32_t qz, int32_t* ids, int32_t max) {
    if (qx < 1 || qy < 1 || qz < 1 || max < 0) return EDP_E_INVALID;
    int n = 0;
    for (int t = 0; t < NUM_ALL_TILES; ++t) {
        if (kind_of(t) != TK_3D || !fits(t, qx, qy, qz)) continue;
        if (ids && n < max) ids[n] = t;
        ++n;
    }
    return n;
}

int32_t edp_wide_tiles_3d(int32_t qx, int32_t qy, int32_t qz, int32_t* ids, int32_t max) {
    if (qx < 1 || qy < 1 || qz < 1 || max < 0) return EDP_E_INVALID;
    int n = 0;
    for (int t = 0; t < NUM_ALL_TILES; ++t) {
        if (kind_of(t) != TK_WIDE3 || !fits(t, qx, qy, qz)) continue;
        if (ids && n < max) ids[n] = t;
        ++n;
    }
    return n;
}

edp_status edp_tile_depth(int32_t tile, int32_t* kz) {
    if (kind_of(tile) == TK_NONE || !kz) return EDP_E_INVALID;
    *kz = kTiles[tile].kz;
    return EDP_OK;
}

edp_status edp_tile_info(int32_t tile, int32_t* px, int32_t* kx, int32_t* py, int32_t* ky) {
    if (kind_of(tile) == TK_NONE || !px || !kx || !py || !ky) return EDP_E_INVALID;
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
        case EDP_E_TIMEOUT: return "a scan's bounded wait gave up (results invalid)";
    }
    return "unknown status";
}

}  // extern "C"
