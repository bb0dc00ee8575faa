/*
 * edp.h -- C ABI of the MI355X (gfx950) scanline-DP / EDP energy minimiser.
 *
 * Method: M. G. Mozerov, "Extended Dynamic Programming and Fast
 * Multidimensional Search Algorithm for Energy Minimization in Stereo and
 * Motion" (arXiv 1410.7922).
 *
 *   Energy (Sec. 2, eq. GE_objective_function with the truncated prior of
 *   eq. Smooth_value_t; f(a) = |a| for EDP_PRIOR_LINEAR, f(a) = a^2 for
 *   EDP_PRIOR_SQUARED, the two priors of Sec. 5.1):
 *       E(v) = sum_x C(x, v(x)) + sum over neighbour pairs (x, x') V(v(x') - v(x))
 *       V(u) = lambda * (min(f(ux), f(T)) + min(f(uy), f(T)))   trunc_mode EDP_TRUNC_PER_DIM
 *       V(u) = lambda * min(f(ux) + f(uy), f(T))                trunc_mode EDP_TRUNC_JOINT
 *   with a third term in uz for a three-dimensional disparity space (Sec. 2
 *   defines the energy for a disparity vector of any dimension R).
 *   Minimum search (Sec. 2, eq. M_strf): M(h)(v) = min_v' h(v') + V(v - v'),
 *   never by the O(Q^2) scan: for the linear prior by the linear recursive
 *   minimum search of Sec. 3.2 (two passes per label dimension plus the clip
 *   of eq. L_dec7), for the squared prior by the general one of Sec. 3.1 (a
 *   window minimum over |u| < T per label dimension plus the clip of
 *   eq. M_decmp, 2T - 1 candidates per label and dimension).
 *
 * Conventions shared by every entry point
 *   - Cost volume: dense, row-major C[y][x][q], int16 or int32, caller-owned
 *     device memory, aligned to the element size.  Labels are flat and 0-based:
 *     q = (vz * qy + vy) * qx + vx (stereo: qy = 1; two label dimensions:
 *     qz = 1, so q = vy * qx + vx).
 *   - All d_* pointers are device pointers owned by the caller; the library
 *     allocates nothing.  Scratch memory is the caller's workspace d_ws of at
 *     least edp_workspace_size() bytes, 256-byte aligned; its contents are
 *     undefined between calls and two calls in flight must not share it.
 *   - stream is a hipStream_t (NULL = the default stream).  Calls only
 *     enqueue work: outputs are valid after the stream is synchronised.
 *   - Errors are returned, never thrown.  Argument errors are detected on the
 *     host before anything is enqueued; nothing is written on error.
 *   - Integer arithmetic only: results are bit-exact and deterministic.
 *     Every argmin takes the smallest flat label.
 *   - Label spaces (at most 4096 labels): the EDP scans hold a vertex's
 *     labels on one lane tile (edp_tiles()) or, for two label dimensions
 *     with a window search (T <= 3), on a wide tile of several wavefronts
 *     (edp_wide_tiles()).  Supported: one label dimension up to 256 labels
 *     (qy == 1); two dimensions up to 32 x 32 with any T, up to 64 x 64
 *     (64 x 32, 32 x 64) with T <= 3; three dimensions up to 8 x 8 x 8
 *     (edp_tiles_3d(), and with T <= 3 also edp_wide_tiles_3d()).  The
 *     scanline DP calls take the single-wavefront
 *     tiles only (256 labels in one dimension, 32 x 32 in two).  Other label
 *     spaces return EDP_E_UNSUPPORTED (edp_dsi and edp_energy take any label
 *     space of up to 4096 labels).
 *     Three label dimensions (qz > 1) are taken by edp_solve, edp_batch_*,
 *     edp_energy and edp_workspace_size with EDP_OP_EDP; the scanline DP
 *     calls and the label-window solve return EDP_E_UNSUPPORTED for them.
 *   - Bounded waits: the EDP scans of one solve run as a pipelined wavefront
 *     whose workgroups wait for each other.  Every such wait gives up after a
 *     bounded number of polls (of the order of a second) instead of hanging the
 *     device.  A solve whose wait gave up has invalid labels; it sets its
 *     status word (d_status) to EDP_E_TIMEOUT and its energy word to INT64_MIN.
 *     The call itself has returned EDP_OK by then (the wait happens on the
 *     device), so callers that need to know read the status word after the
 *     stream is synchronised.
 */
#ifndef EDP_H
#define EDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EDP_OK = 0,
    EDP_E_INVALID = -1,     /* bad argument: null pointer, size, dtype, mode, ... */
    EDP_E_RANGE = -2,       /* the int32 range guard failed for these parameters */
    EDP_E_WORKSPACE = -3,   /* workspace missing, misaligned or too small */
    EDP_E_HIP = -4,         /* a HIP runtime call or kernel launch failed */
    EDP_E_UNSUPPORTED = -5, /* valid problem outside what the library implements */
    EDP_E_TIMEOUT = -6      /* device status word only: a scan's bounded wait gave up */
} edp_status;

typedef enum { EDP_I16 = 1, EDP_I32 = 2 } edp_dtype;
typedef enum { EDP_TRUNC_PER_DIM = 0, EDP_TRUNC_JOINT = 1 } edp_trunc_mode;
typedef enum { EDP_PRIOR_LINEAR = 0, EDP_PRIOR_SQUARED = 1 } edp_prior;
typedef enum { EDP_OP_DP = 0, EDP_OP_EDP = 1, EDP_OP_DP_MARGINALS = 2 } edp_op;

/* One energy-minimisation instance (Sec. 2). */
typedef struct {
    int32_t width;       /* W = x_max >= 1 */
    int32_t height;      /* H = y_max >= 1 */
    int32_t qx;          /* labels along the first label dimension, >= 1 */
    int32_t qy;          /* labels along the second label dimension, >= 1 (1 for stereo) */
    int32_t dtype;       /* edp_dtype of the cost volume */
    int32_t trunc_mode;  /* edp_trunc_mode; the two modes coincide with one label dimension */
    int32_t lambda;      /* prior weight, 0 <= lambda <= 65535 */
    int32_t trunc;       /* truncation threshold T (the paper's g), 1 <= T <= 4096 */
    int32_t iterations;  /* EDP iterations j >= 1 of Algorithm 1 (ignored by the DP) */
    int32_t cost_bound;  /* promise |C| <= cost_bound; 0 = the dtype's range (int16 only) */
    int32_t prior;       /* edp_prior: f(a) = |a| (0) or a^2 (1) */
    int32_t qz;          /* labels along a third label dimension; 0 or 1 = none (R <= 2) */
} edp_problem;

/* Optional tuning of the launch (results never depend on it).  NULL, or a
 * zero / negative field, selects the built-in choice:
 *   tile   lane tile mapping labels to lanes (edp_tiles(), or for the EDP
 *          scans also edp_wide_tiles(), edp_tiles_3d() and
 *          edp_wide_tiles_3d(); -1 automatic)
 *   chunk  EDP columns a workgroup hands to the next one between two
 *          progress publications, at least (rounded up to a power of two);
 *          only where the hand-off publishes column counts (wavefronts of
 *          one scanline, or instances whose tagged hand-off rows would
 *          exceed 32 MB)
 *   split  1: every lane runs both minimum searches of a scan step;
 *          2: the two searches run on two halves of the vertex's lanes
 *   waves  compute wavefronts per EDP workgroup (1..6), handing rows over in
 *          LDS; every workgroup has two more wavefronts that move the rows
 *          between workgroups.  Wide tiles: scanlines per workgroup (at most
 *          8 / (its wavefronts per vertex)); rows go between workgroups as
 *          tagged words
 *   fuse   EDP scans per launch: 1, or 2 (P1 with P2, P3 with P4: the two
 *          scans of a pair sweep the rows in the same order, so the second
 *          follows the first a few rows behind inside one launch)
 * events (nullable): caller-created hipEvent_t handles recorded on the call's
 * stream so the caller can time kernels: edp_solve records events[2l] before
 * and events[2l+1] after its l-th scan launch (l < n_events / 2);
 * edp_dp_scanline records events[0], [1] around the forward sweep and
 * events[2], [3] around the backtracking.  Handles past n_events are unused. */
typedef struct {
    int32_t tile;        /* tile id from edp_tiles(), or -1 for automatic */
    int32_t chunk;       /* EDP columns per progress publication, 0 = automatic */
    int32_t split;       /* 1 or 2, 0 = automatic */
    int32_t waves;       /* 1..6, 0 = automatic */
    int32_t fuse;        /* 1 or 2, 0 = automatic */
    void* const* events; /* nullable, see above */
    int32_t n_events;    /* number of handles in events */
} edp_tuning;

/* Workspace bytes needed by op (edp_op) for prob under tuning (nullable). */
edp_status edp_workspace_size(const edp_problem* prob, int32_t op, const edp_tuning* tuning,
                              size_t* bytes);

/*
 * Independent scanline DP (Sec. 2 eq. One_d: vertical prior taken as zero).
 * Every row y is a chain solved exactly by the recursion of eq. base,
 * S(0, v) = C(0, v), S(x+1, v) = C(x+1, v) + M(S(x, .))(v) (zero boundary of
 * Sec. 4.1 eq. DP_1D_2); its energy is min_v S(W-1, v) and its labels are read
 * back from the stored optimal choice indexes (Sec. 4.1).  Among optimal
 * labellings the reverse-lexicographically smallest one is returned.
 *   d_cost        [H][W][Q] cost volume
 *   d_labels      [H][W] int32 output labels
 *   d_row_energy  [H] int64 output row energies (nullable)
 *   d_energy      [1] int64 output: sum of the row energies (nullable)
 */
edp_status edp_dp_scanline(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                           int32_t* d_labels, int64_t* d_row_energy, int64_t* d_energy,
                           void* d_ws, size_t ws_bytes, void* stream);

/*
 * Scanline DP by min-marginals (Sec. 4.1, eqs. DP_1D_3 and DP_1D_5): for every
 * row, a forward recursion S_1(x) = C(x) + M(S_1(x-1)) from S_1(0) = C(0) and a
 * backward one S_-1(x) = C(x) + M(S_-1(x+1)) from S_-1(W-1) = C(W-1) give the
 * marginal S_Omega(x, v) = M(S_1(x-1))(v) + C(x, v) + M(S_-1(x+1))(v) (terms
 * off the row are 0); each label is the smallest argmin of its own column's
 * marginal, with no stored choice indexes and no walk back.  min_v S_Omega(x, v)
 * equals the row optimum at every x; the labels are the DP's optimal labelling
 * wherever that is unique, and otherwise may combine several optimal labellings
 * (their energy, from edp_energy, can then exceed the row optimum).  The
 * forward terms are stored in 16 bits: problems whose clip distance lambda f(T)
 * (twice that per-dimension in two label dimensions) exceeds 65535 return
 * EDP_E_RANGE.  Workspace: edp_workspace_size with EDP_OP_DP_MARGINALS.
 * tuning: tile as for the DP; events[0], [1] around the forward sweep, [2],
 * [3] around the backward sweep.
 *   d_labels      [H][W] int32 output labels
 *   d_marginal    [H][W][Q] int32 output S_Omega(x, v) - min_v S_Omega(x, v) (nullable)
 *   d_row_energy  [H] int64 output row optima (nullable)
 *   d_energy      [1] int64 output: their sum (nullable)
 */
edp_status edp_dp_marginals(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                            int32_t* d_labels, int32_t* d_marginal, int64_t* d_row_energy, int64_t* d_energy,
                            void* d_ws, size_t ws_bytes, void* stream);

/*
 * Extended DP (Sec. 4.2, Algorithm 1 steps 3-5) on the 4-connected grid:
 * prob->iterations rounds of the scans P1..P4 of eq. DP_2D_base (with the data
 * cost added and S/2 taken as floor division), then the marginal of eq. DP_2D_1
 * and its smallest argmin (eq. DP_2D_2).
 *   d_labels  [H][W] int32 output labels
 *   d_energy  [1] int64 output: 4-connected energy of d_labels (nullable);
 *             INT64_MIN when a scan's bounded wait gave up
 *   d_status  [1] int32 output (nullable): EDP_OK, or EDP_E_TIMEOUT when a
 *             scan's bounded wait gave up (labels and energy are then invalid)
 */
edp_status edp_solve(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                     int32_t* d_labels, int64_t* d_energy, int32_t* d_status, void* d_ws,
                     size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): edp_solve with its
 * workspace in a static device array of EDP_STATIC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends.  The call
 * allocates nothing.  Problems whose EDP workspace (edp_workspace_size with
 * EDP_OP_EDP and the same tuning) exceeds the array return EDP_E_WORKSPACE
 * before anything is enqueued; for example stereo 384 x 288 with 32
 * disparities (about 60 MB) fits.  stream must belong to the current device
 * (EDP_E_INVALID otherwise).  Every call on one GPU uses that GPU's single
 * array, so calls that overlap on one GPU (on different streams or from
 * different host threads) race and give wrong results; calls one after another
 * on one stream are fine.  Arguments and results as for edp_solve.
 */
#define EDP_STATIC_SCRATCH_BYTES (64u << 20)
edp_status edp_solve_static(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                            int32_t* d_labels, int64_t* d_energy, int32_t* d_status, void* stream);

/*
 * Label-window EDP: the EDP of edp_solve restricted, at every vertex x, to the
 * win x win box of labels centred on d_centers[y][x] = (cx, cy) -- by
 * definition the plain EDP on the cost volume with every label outside the
 * vertex's box given an infinite cost.  Each vertex keeps its box in a frame
 * of 8 x 8 labels and every sum handed to a neighbour is evaluated in the
 * neighbour's frame, so the work per vertex does not grow with Q.  win odd,
 * 1 <= win <= 8, boxes inside the label space (win/2 <= cx < qx - win/2, same
 * for cy); qx - win <= 127 and qy - win <= 127 (the shifts between
 * neighbouring frames are kept in 8 bits); int32 costs; the truncated linear
 * prior only (EDP_E_UNSUPPORTED otherwise).  The energy is that of the labels
 * on the full cost; d_energy and d_status as for edp_solve.
 * tuning: tile must be -1 or 13 (the 8 x 8 lane tile, one label per lane),
 *         split 1; waves, chunk, fuse as for edp_solve.
 *   d_centers [H][W][2] int32;  d_labels [H][W] int32 labels of the full space
 */
edp_status edp_window_workspace_size(const edp_problem* prob, int32_t win, const edp_tuning* tuning,
                                     size_t* bytes);
edp_status edp_solve_windowed(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                              const int32_t* d_centers, int32_t win, int32_t* d_labels, int64_t* d_energy,
                              int32_t* d_status, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Batches: many independent EDP instances (Algorithm 1 each, any mix of grid
 * sizes, label spaces, dtypes and parameters) solved by shared persistent
 * launches.  Instances with the same launch shape (tile, cost kind, split,
 * waves, chunk, fuse, iterations) form a class; each scan launch of a class
 * walks a work queue over (scan, instance, workgroup band), longest instance
 * first.  Classes run on library-owned streams forked from and joined back to
 * the caller's stream.  Results are identical to edp_solve on each instance.
 */
typedef struct {
    edp_problem problem;
    const void* d_cost;    /* [H][W][Q] cost volume */
    int32_t* d_labels;     /* [H][W] int32 output labels */
    int64_t* d_energy;     /* [1] int64 output: 4-connected energy (nullable; INT64_MIN on timeout) */
    int32_t* d_status;     /* [1] int32 output status word as for edp_solve (nullable) */
    edp_tuning tuning;     /* launch shape of this instance (events ignored) */
} edp_batch_item;

typedef struct edp_batch_plan edp_batch_plan;   /* opaque, host memory */

/* Workspace bytes of a batch: every instance's arrays plus a descriptor table. */
edp_status edp_batch_workspace_size(int32_t n, const edp_batch_item* items, size_t* bytes);

/*
 * Validate the batch, group it into classes and write the descriptor table
 * into d_ws (a copy on stream that this call waits for: the one synchronising
 * step, done once per batch layout).  The plan keeps d_ws and the item
 * pointers; it stays valid until edp_batch_plan_destroy.  Errors leave *plan
 * untouched.
 */
edp_status edp_batch_plan_create(int32_t n, const edp_batch_item* items, void* d_ws, size_t ws_bytes,
                                 void* stream, edp_batch_plan** plan);

/*
 * Enqueue one solve of every instance of the plan on stream.  Only kernel
 * launches and event records/waits are enqueued (no copies, no memsets, no
 * allocation), so the call can be captured into a hipGraph and replayed.
 * Solves of one plan must not overlap: they share its workspace.
 */
edp_status edp_batch_solve(const edp_batch_plan* plan, void* stream);

/* Classes and kernel launches of one edp_batch_solve (either nullable). */
edp_status edp_batch_plan_info(const edp_batch_plan* plan, int32_t* n_classes, int32_t* n_launches);

/* Release the plan's host memory, streams and events (NULL is ignored).  The
 * caller first synchronises every stream that ran the plan's solves. */
void edp_batch_plan_destroy(edp_batch_plan* plan);

/*
 * Data cost (DSI) formation, Sec. 2 eq. Cost_value:
 *   C(x, v) = min(|I1(x + v) - I0(x)|^l2, cmax),  l2 = 1 or 2,
 * or, with a third image d_i2 (the composite three-view cost of Sec. 5.1
 * eq. Cost_cmp, for occlusion handling):
 *   C(x, v) = min(C_{0->1}(x, v), C_{0->2}(x, -v)).
 * Label q = iy * qx + ix has the displacement v = (ox + sx * ix, oy + sy * iy),
 * sx, sy = +1 or -1: rectified stereo with I1 the right image is qy = 1,
 * ox = 0, sx = -1; motion within [-r, r]^2 is ox = oy = -r, sx = sy = 1.  A
 * displaced position outside the image costs cmax for that view; |ox|, |oy| <=
 * 16384.
 *   d_i0, d_i1  [H][W] uint8 images (device); d_i2 the third view or NULL
 *   dtype       EDP_I16 (0 <= cmax <= 32767) or EDP_I32 (cmax >= 0)
 *   d_cost      [H][W][qx*qy] output, aligned to its element size
 * Only a kernel launch is enqueued; no workspace.
 */
edp_status edp_dsi(const uint8_t* d_i0, const uint8_t* d_i1, const uint8_t* d_i2, int32_t width, int32_t height,
                   int32_t qx, int32_t qy, int32_t ox, int32_t oy, int32_t sx, int32_t sy, int32_t l2, int32_t cmax,
                   int32_t dtype, void* d_cost, void* stream);

/*
 * Energy of a labelling (Sec. 2 eq. GE_objective_function).
 *   grid4      0: horizontal pairs only (the scanline energy), 1: 4-connected
 *   d_labels   [H][W] int32 labels; labels outside [0, Q) contribute nothing
 *   d_energy   [1] int64 output
 *   d_invalid  [1] int64 output, count of labels outside [0, Q) (nullable)
 */
edp_status edp_energy(const edp_problem* prob, const void* d_cost, const int32_t* d_labels,
                      int32_t grid4, int64_t* d_energy, int64_t* d_invalid, void* stream);

/* Lane tiles usable for a (qx, qy) label space.  Writes up to max ids into ids
 * (nullable) and returns how many exist; a negative value is an edp_status. */
int32_t edp_tiles(int32_t qx, int32_t qy, int32_t* ids, int32_t max);

/* Wide-vertex tiles of the EDP scans usable for a (qx, qy) label space (two
 * label dimensions, truncation T <= 3 so the minimum search is the general RMS
 * window of at most two steps per side, Sec. 3.1).  A vertex takes py / 4
 * wavefronts, each holding 4 ky label rows of 16 kx labels; its scans exchange
 * the label rows at slab edges through LDS at every step (Sec. 3 eq. M_decmp:
 * one window per label dimension).  Same return convention as edp_tiles(). */
int32_t edp_wide_tiles(int32_t qx, int32_t qy, int32_t* ids, int32_t max);

/* Lane tiles of the EDP scans usable for a (qx, qy, qz) label space with three
 * label dimensions.  Lane (px, py) of a vertex holds its kx * ky labels at each
 * of the kz labels of the third dimension, so the operator of that dimension
 * (one per label dimension, Sec. 3 eq. M_decmp) works inside the lane.  Same
 * return convention as edp_tiles(). */
int32_t edp_tiles_3d(int32_t qx, int32_t qy, int32_t qz, int32_t* ids, int32_t max);

/* Wide-vertex tiles of the EDP scans usable for a (qx, qy, qz) label space with
 * three label dimensions and truncation T <= 3 (the general RMS window of at
 * most two steps per side, Sec. 3.1).  A vertex of up to 8 x 8 x kz labels
 * (edp_tile_depth()) takes several wavefronts, each holding every (x, y) label
 * at a few labels of the third dimension: the operators along x and y work
 * inside the wavefront, the one along z exchanges the wavefronts' labels through
 * LDS at every step (Sec. 3 eq. M_decmp).  Same return convention as
 * edp_tiles(). */
int32_t edp_wide_tiles_3d(int32_t qx, int32_t qy, int32_t qz, int32_t* ids, int32_t max);

/* Shape of a tile (edp_tiles(), edp_wide_tiles(), edp_tiles_3d() or
 * edp_wide_tiles_3d()): lanes px * py per cell, labels kx * ky per lane at each
 * of its edp_tile_depth() labels along the third dimension (for the wide tiles
 * the labels of all wavefronts of a vertex: 4 py wavefronts of 16 px lanes in
 * two dimensions; 8 x 8 lanes per wavefront, the edp_tile_depth() labels along
 * z spread over the wavefronts in three). */
edp_status edp_tile_info(int32_t tile, int32_t* px, int32_t* kx, int32_t* py, int32_t* ky);

/* Labels kz along the third label dimension that a tile holds (every lane of
 * a tile of edp_tiles_3d(); all wavefronts of a vertex together for a tile of
 * edp_wide_tiles_3d(); 1 for the tiles of one or two label dimensions). */
edp_status edp_tile_depth(int32_t tile, int32_t* kz);

/* Static text for a status code. */
const char* edp_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* EDP_H */
