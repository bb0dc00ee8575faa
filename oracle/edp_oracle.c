/*
 * Plain C oracle for scanline DP and EDP (Mozerov, arXiv 1410.7922).
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library.  It shares no code with the
 * GPU library and is written from the paper's definitions:
 *
 *   labels   flat q = (vz * qy + vy) * qx + vx over R = 1, 2 or 3 label
 *            dimensions (qz = 1 below three; Sec. 2 defines the search for any R).
 *   V(u)     truncated prior, Sec. 2 eq. Smooth_value_t with f(|a|) = |a|
 *            (prior 0, truncated linear) or f(|a|) = a^2 (prior 1, truncated
 *            squared, l_1 = 2 of Sec. 5.1); mode 0 truncates each label
 *            dimension, mode 1 the summed distance.
 *   M(h)(v)  = min_v' h(v') + V(v - v')       Sec. 2 eq. M_strf
 *            search 0: straightforward search over all v' (SFMS, the definition)
 *            search 1: the linear RMS passes of Sec. 3.2 (eqs. L_dec3, L_dec5
 *                      read as the mirror of L_dec3, L_dec6, clip of L_dec7);
 *                      truncated linear prior only
 *            search 2: the general RMS of Sec. 3.1: per label dimension the
 *                      window minimum over |u_r| < g of eq. M_decmp1 (with the
 *                      penalty lambda f(|u_r|) inside the minimum), then the
 *                      clip of eq. M_decmp (per line in mode 0).
 *            Searches 1 and 2 take the dimensions in the order x, y, z.
 *   DP       S(0)=C(0), S(x+1)=C(x+1)+M(S(x))  Sec. 2 eq. base, Sec. 4.1
 *   EDP      Sec. 4.2 eq. DP_2D_base with C added, S/2 as floor division,
 *            scans P1..P4 in place, eq. DP_2D_1 marginal, eq. DP_2D_2 argmin.
 *   windowed EDP: the same on a cost volume masked by a sentinel outside a
 *            per-vertex label box (the definition of the label-window solve).
 *   volume EDP (D = 3): eq. DP_2D_base and eq. DP_2D_1 in their general form,
 *            K = {+-x, +-y, +-z}, S/3 as floor division, the eight raster scans
 *            of a volume (x innermost; x order alternating fastest, then y,
 *            then z), 6-connected energy.
 *
 * All sums are computed and stored in int64 and range-checked against int32
 * (the check's failure is reported, never wrapped).  Single threaded.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARGS -1
#define OR_E_RANGE -2
#define OR_E_NOMEM -3

typedef struct {
    int qx, qy, qz, q, lam, trunc, mode, prior;
} prior_t;

static prior_t make_prior(int qx, int qy, int qz, int lam, int trunc, int mode, int prior) {
    prior_t p = {qx, qy, qz, qx * qy * qz, lam, trunc, mode, prior};
    return p;
}

static int64_t iabs64(int64_t a) { return a < 0 ? -a : a; }
static int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

/* f of eq. Smooth_value_t */
static int64_t prior_f(const prior_t *p, int64_t a) { return p->prior == 1 ? a * a : iabs64(a); }

/* coordinate r (0 x, 1 y, 2 z) of flat label v */
static int coord(const prior_t *p, int v, int r) {
    if (r == 0) return v % p->qx;
    if (r == 1) return (v / p->qx) % p->qy;
    return v / (p->qx * p->qy);
}

static int64_t prior_v(const prior_t *p, int v, int w) {
    int64_t fg = prior_f(p, p->trunc), sum = 0, trunc_each = 0;
    for (int r = 0; r < 3; ++r) {
        int64_t f = prior_f(p, (int64_t)coord(p, v, r) - coord(p, w, r));
        sum += f;
        trunc_each += imin64(f, fg);
    }
    if (p->mode == 0) return (int64_t)p->lam * trunc_each;
    return (int64_t)p->lam * imin64(sum, fg);
}

/* Lines of the label grid along dimension r: length n, label stride st; a line starts
 * at every label whose coordinate r is 0. */
static void line_shape(const prior_t *p, int r, int *n, int *st) {
    *n = r == 0 ? p->qx : r == 1 ? p->qy : p->qz;
    *st = r == 0 ? 1 : r == 1 ? p->qx : p->qx * p->qy;
}

/* M by straightforward search; arg (nullable) receives the smallest minimising v'. */
static void msearch_sfms(const prior_t *p, const int64_t *h, int64_t *out, int32_t *arg) {
    for (int v = 0; v < p->q; ++v) {
        int64_t best = h[0] + prior_v(p, v, 0);
        int bi = 0;
        for (int w = 1; w < p->q; ++w) {
            int64_t t = h[w] + prior_v(p, v, w);
            if (t < best) { best = t; bi = w; }
        }
        out[v] = best;
        if (arg) arg[v] = bi;
    }
}

/* One line of L_r: forward S+ (eq. L_dec3), backward S- over strictly larger
 * labels with S-(last) = +inf (eq. L_dec5, mirrored), comparison (eq. L_dec6). */
static void lrms_line(int64_t *line, int n, int stride, int64_t lam, int64_t *plus, int64_t *minus) {
    plus[0] = line[0];
    for (int v = 1; v < n; ++v) plus[v] = imin64(plus[v - 1] + lam, line[(size_t)v * stride]);
    int have = 0;
    for (int v = n - 2; v >= 0; --v) {
        int64_t nxt = line[(size_t)(v + 1) * stride];
        if (have) nxt = imin64(nxt, minus[v + 1]);
        minus[v] = nxt + lam;
        have = 1;
    }
    for (int v = 0; v < n; ++v) {
        int64_t r = plus[v];
        if (v < n - 1) r = imin64(r, minus[v]);
        line[(size_t)v * stride] = r;
    }
}

static void msearch_lrms(const prior_t *p, const int64_t *h, int64_t *out, int64_t *scratch) {
    int64_t *plus = scratch, *minus = scratch + 4096;
    int64_t lam = p->lam, clipd = (int64_t)p->lam * p->trunc;
    int64_t gmin = h[0];
    for (int v = 0; v < p->q; ++v) { out[v] = h[v]; if (h[v] < gmin) gmin = h[v]; }
    for (int r = 0; r < 3; ++r) {                  /* dimensions x, y, z in turn */
        int n, st;
        line_shape(p, r, &n, &st);
        if (r > 0 && n == 1) continue;
        for (int v0 = 0; v0 < p->q; ++v0) {
            if (coord(p, v0, r) != 0) continue;
            int64_t *line = out + v0;
            int64_t lmin = line[0];
            for (int i = 1; i < n; ++i) lmin = imin64(lmin, line[(size_t)i * st]);
            lrms_line(line, n, st, lam, plus, minus);
            if (p->mode == 0)
                for (int i = 0; i < n; ++i) line[(size_t)i * st] = imin64(line[(size_t)i * st], lmin + clipd);
        }
    }
    if (p->mode == 1)
        for (int v = 0; v < p->q; ++v) out[v] = imin64(out[v], gmin + clipd);
}

/* One line of M-bar_r (eq. M_decmp1): out(v) = min over |u| < g, v - u on the line, of
 * line(v - u) + lambda f(|u|).  out must not alias line. */
static void grms_line(const prior_t *p, const int64_t *line, int n, int stride, int64_t *out) {
    for (int v = 0; v < n; ++v) {
        int64_t best = line[(size_t)v * stride];
        for (int u = 1; u < p->trunc; ++u) {
            int64_t pen = (int64_t)p->lam * prior_f(p, u);
            if (v - u >= 0) best = imin64(best, line[(size_t)(v - u) * stride] + pen);
            if (v + u < n) best = imin64(best, line[(size_t)(v + u) * stride] + pen);
        }
        out[v] = best;
    }
}

static void msearch_grms(const prior_t *p, const int64_t *h, int64_t *out, int64_t *scratch) {
    int64_t *tmp = scratch;
    int64_t clipd = (int64_t)p->lam * prior_f(p, p->trunc);
    int64_t gmin = h[0];
    for (int v = 0; v < p->q; ++v) { out[v] = h[v]; if (h[v] < gmin) gmin = h[v]; }
    for (int r = 0; r < 3; ++r) {                  /* dimensions x, y, z in turn */
        int n, st;
        line_shape(p, r, &n, &st);
        if (r > 0 && n == 1) continue;
        for (int v0 = 0; v0 < p->q; ++v0) {
            if (coord(p, v0, r) != 0) continue;
            int64_t *line = out + v0;
            int64_t lmin = line[0];
            for (int i = 1; i < n; ++i) lmin = imin64(lmin, line[(size_t)i * st]);
            grms_line(p, line, n, st, tmp);
            for (int i = 0; i < n; ++i)
                line[(size_t)i * st] = p->mode == 0 ? imin64(tmp[i], lmin + clipd) : tmp[i];
        }
    }
    if (p->mode == 1)
        for (int v = 0; v < p->q; ++v) out[v] = imin64(out[v], gmin + clipd);
}

static void msearch(const prior_t *p, int search, const int64_t *h, int64_t *out, int64_t *scratch) {
    if (search == 1) msearch_lrms(p, h, out, scratch);
    else if (search == 2) msearch_grms(p, h, out, scratch);
    else msearch_sfms(p, h, out, NULL);
}

static int check_args(int W, int H, int qx, int qy, int qz, int lam, int trunc, int mode, int prior, int search) {
    if (W < 1 || H < 1 || qx < 1 || qy < 1 || qz < 1 || qx > 4096 || qy > 4096 || qz > 4096 ||
        (int64_t)qx * qy * qz > 4096)
        return 0;
    if (lam < 0 || trunc < 1 || trunc > 4096 || (mode != 0 && mode != 1)) return 0;
    if (prior != 0 && prior != 1) return 0;
    if (search < 0 || search > 2 || (search == 1 && prior != 0)) return 0;
    return 1;
}

/* Energy of eq. GE_objective_function; grid4 = 0: rows only, 1: 4-connected. */
int64_t oracle_energy(int W, int H, int qx, int qy, int qz, int lam, int trunc, int mode, int prior, int grid4,
                      const int32_t *cost, const int32_t *labels) {
    prior_t p = make_prior(qx, qy, qz, lam, trunc, mode, prior);
    int64_t e = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int l = labels[(size_t)y * W + x];
            e += cost[((size_t)y * W + x) * p.q + l];
            if (x + 1 < W) e += prior_v(&p, labels[(size_t)y * W + x + 1], l);
            if (grid4 && y + 1 < H) e += prior_v(&p, labels[(size_t)(y + 1) * W + x], l);
        }
    return e;
}

/* Scanline DP over every row.  search 0: SFMS with stored choice indexes;
 * search 1 (LRMS) or 2 (GRMS): the values, and at backtracking the choice index
 * at the chosen label is found by direct search over the stored S(x-1) (the
 * same argmin). */
int oracle_dp_scanline(int W, int H, int qx, int qy, int qz, int lam, int trunc, int mode, int prior, int search,
                       const int32_t *cost, int32_t *labels, int64_t *row_energy, int64_t *total) {
    if (!check_args(W, H, qx, qy, qz, lam, trunc, mode, prior, search)) return OR_E_ARGS;
    prior_t p = make_prior(qx, qy, qz, lam, trunc, mode, prior);
    int Q = p.q;
    int64_t *S = malloc(sizeof(int64_t) * (size_t)W * Q);
    int64_t *m = malloc(sizeof(int64_t) * Q);
    int64_t *scratch = malloc(sizeof(int64_t) * 8192);
    int32_t *ptr = malloc(sizeof(int32_t) * (size_t)W * Q);
    if (!S || !m || !scratch || !ptr) { free(S); free(m); free(scratch); free(ptr); return OR_E_NOMEM; }
    int64_t tot = 0;
    for (int y = 0; y < H; ++y) {
        const int32_t *c = cost + (size_t)y * W * Q;
        for (int v = 0; v < Q; ++v) S[v] = c[v];
        for (int x = 1; x < W; ++x) {
            if (search != 0) msearch(&p, search, S + (size_t)(x - 1) * Q, m, scratch);
            else msearch_sfms(&p, S + (size_t)(x - 1) * Q, m, ptr + (size_t)x * Q);
            for (int v = 0; v < Q; ++v) S[(size_t)x * Q + v] = c[(size_t)x * Q + v] + m[v];
        }
        const int64_t *last = S + (size_t)(W - 1) * Q;
        int bi = 0;
        for (int v = 1; v < Q; ++v) if (last[v] < last[bi]) bi = v;
        row_energy[y] = last[bi];
        tot += last[bi];
        int32_t *lab = labels + (size_t)y * W;
        lab[W - 1] = bi;
        for (int x = W - 1; x > 0; --x) {
            int v = lab[x];
            if (search != 0) {
                const int64_t *prev = S + (size_t)(x - 1) * Q;
                int64_t best = prev[0] + prior_v(&p, v, 0);
                int b = 0;
                for (int w = 1; w < Q; ++w) {
                    int64_t t = prev[w] + prior_v(&p, v, w);
                    if (t < best) { best = t; b = w; }
                }
                lab[x - 1] = b;
            } else {
                lab[x - 1] = ptr[(size_t)x * Q + v];
            }
        }
    }
    *total = tot;
    free(S); free(m); free(scratch); free(ptr);
    return OR_OK;
}

static int64_t floor_half(int64_t s) { return s >= 0 ? s / 2 : -((-s + 1) / 2); }

/* direction k: 0 +x, 1 -x, 2 +y, 3 -y; predecessor x_k = x - sgn(k) e_|k| */
static const int KDX[4] = {1, -1, 0, 0};
static const int KDY[4] = {0, 0, 1, -1};
static const int KOPP[4] = {1, 0, 3, 2};

/* Literal EDP (Algorithm 1 steps 3-5) with an optional label window per vertex.
 *
 * Without a window (centers NULL) this is the plain EDP.  With a window, the
 * cost of every label outside the win x win box centred on centers[y][x] =
 * (cx, cy) is taken as the sentinel SENT, larger than any reachable sum of the
 * in-box labels: the windowed EDP is defined as the plain EDP on that masked
 * cost volume.  Sums are kept in int64; the int32 range check covers the
 * in-box labels only (the out-of-box sums carry the sentinel).  The energy of
 * the result is evaluated with the unmasked cost.
 * marginal_out [H][W][Q] int64 is nullable. */
#define SENT ((int64_t)1 << 40)

static int in_box(const int32_t *centers, int win, int W, int qx, int x, int y, int v) {
    if (!centers) return 1;
    const int32_t *c = centers + ((size_t)y * W + x) * 2;
    int r = win / 2;
    int vx = v % qx, vy = v / qx;            /* windows are defined on two-dimensional label spaces */
    return vx >= c[0] - r && vx <= c[0] + r && vy >= c[1] - r && vy <= c[1] + r;
}

static int edp_core(int W, int H, int qx, int qy, int qz, int lam, int trunc, int mode, int prior,
                    int iterations, int search, const int32_t *cost, const int32_t *centers, int win,
                    int32_t *labels, int64_t *energy_out, int64_t *max_abs_out, int64_t *marginal_out) {
    if (!check_args(W, H, qx, qy, qz, lam, trunc, mode, prior, search) || iterations < 0) return OR_E_ARGS;
    if (centers && (win < 1 || win % 2 == 0 || qz != 1)) return OR_E_ARGS;
    prior_t p = make_prior(qx, qy, qz, lam, trunc, mode, prior);
    int Q = p.q;
    size_t cells = (size_t)W * H;
    int64_t *S = calloc((size_t)4 * cells * Q, sizeof(int64_t));
    int64_t *h = malloc(sizeof(int64_t) * Q);
    int64_t *m = malloc(sizeof(int64_t) * 4 * Q);
    int64_t *acc = malloc(sizeof(int64_t) * Q);
    int64_t *scratch = malloc(sizeof(int64_t) * 8192);
    int64_t *nw = malloc(sizeof(int64_t) * 2 * Q);
    if (!S || !h || !m || !acc || !scratch || !nw) {
        free(S); free(h); free(m); free(acc); free(scratch); free(nw);
        return OR_E_NOMEM;
    }
    int64_t maxabs = 0;
    int status = OR_OK;
    /* scans: x order, y order, computed sums */
    const int sx[4] = {1, -1, 1, -1}, sy[4] = {1, 1, -1, -1};
    const int ka[4] = {0, 1, 0, 1}, kb[4] = {2, 2, 3, 3};
    for (int it = 0; it < iterations; ++it) {
        for (int pass = 0; pass < 4; ++pass) {
            for (int yi = 0; yi < H; ++yi) {
                int y = sy[pass] > 0 ? yi : H - 1 - yi;
                for (int xi = 0; xi < W; ++xi) {
                    int x = sx[pass] > 0 ? xi : W - 1 - xi;
                    for (int k = 0; k < 4; ++k) {      /* m_k = M(S_k(x_k) / 2), 0 off grid */
                        int px = x - KDX[k], py = y - KDY[k];
                        int64_t *mk = m + (size_t)k * Q;
                        if (px < 0 || px >= W || py < 0 || py >= H) {
                            for (int v = 0; v < Q; ++v) mk[v] = 0;
                            continue;
                        }
                        const int64_t *sk = S + ((size_t)k * cells + (size_t)py * W + px) * Q;
                        for (int v = 0; v < Q; ++v) h[v] = floor_half(sk[v]);
                        msearch(&p, search, h, mk, scratch);
                    }
                    const int32_t *c = cost + ((size_t)y * W + x) * Q;
                    int comp[2] = {ka[pass], kb[pass]};
                    for (int j = 0; j < 2; ++j) {       /* eq. DP_2D_base with C added */
                        int kp = comp[j];
                        for (int v = 0; v < Q; ++v) {
                            int64_t s = in_box(centers, win, W, qx, x, y, v) ? (int64_t)c[v] : SENT;
                            for (int k = 0; k < 4; ++k)
                                if (k != KOPP[kp]) s += m[(size_t)k * Q + v];
                            s -= m[(size_t)KOPP[kp] * Q + v];
                            nw[(size_t)j * Q + v] = s;
                        }
                    }
                    for (int j = 0; j < 2; ++j) {
                        int64_t *dst = S + ((size_t)comp[j] * cells + (size_t)y * W + x) * Q;
                        for (int v = 0; v < Q; ++v) {
                            int64_t s = nw[(size_t)j * Q + v];
                            if (in_box(centers, win, W, qx, x, y, v)) {
                                if (iabs64(s) > maxabs) maxabs = iabs64(s);
                                if (s > INT32_MAX || s < INT32_MIN) status = OR_E_RANGE;
                            }
                            dst[v] = s;
                        }
                    }
                }
            }
        }
    }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {                   /* eq. DP_2D_1 with C, eq. DP_2D_2 */
            const int32_t *c = cost + ((size_t)y * W + x) * Q;
            for (int v = 0; v < Q; ++v) acc[v] = in_box(centers, win, W, qx, x, y, v) ? (int64_t)c[v] : SENT;
            for (int k = 0; k < 4; ++k) {
                int px = x - KDX[k], py = y - KDY[k];
                if (px < 0 || px >= W || py < 0 || py >= H) continue;
                const int64_t *sk = S + ((size_t)k * cells + (size_t)py * W + px) * Q;
                for (int v = 0; v < Q; ++v) h[v] = floor_half(sk[v]);
                msearch(&p, search, h, m, scratch);
                for (int v = 0; v < Q; ++v) acc[v] += m[v];
            }
            int bi = 0;
            for (int v = 1; v < Q; ++v) if (acc[v] < acc[bi]) bi = v;
            labels[(size_t)y * W + x] = bi;
            if (marginal_out)
                memcpy(marginal_out + ((size_t)y * W + x) * Q, acc, sizeof(int64_t) * Q);
        }
    *energy_out = oracle_energy(W, H, qx, qy, qz, lam, trunc, mode, prior, 1, cost, labels);
    *max_abs_out = maxabs;
    free(S); free(h); free(m); free(acc); free(scratch); free(nw);
    return status;
}

int oracle_edp(int W, int H, int qx, int qy, int qz, int lam, int trunc, int mode, int prior, int iterations,
               int search, const int32_t *cost, int32_t *labels, int64_t *energy_out,
               int64_t *max_abs_out, int64_t *marginal_out) {
    return edp_core(W, H, qx, qy, qz, lam, trunc, mode, prior, iterations, search, cost, NULL, 1, labels,
                    energy_out, max_abs_out, marginal_out);
}

/* Windowed EDP: centers [H][W][2] (cx, cy) label coordinates, odd window side win. */
int oracle_edp_window(int W, int H, int qx, int qy, int lam, int trunc, int mode, int prior, int iterations,
                      int search, const int32_t *cost, const int32_t *centers, int win,
                      int32_t *labels, int64_t *energy_out, int64_t *max_abs_out) {
    if (!centers) return OR_E_ARGS;
    return edp_core(W, H, qx, qy, 1, lam, trunc, mode, prior, iterations, search, cost, centers, win, labels,
                    energy_out, max_abs_out, NULL);
}

/* M on a batch of n vectors h[n][Q] (search 0: SFMS with arg (nullable); 1: LRMS; 2: GRMS). */
int oracle_min_search(int qx, int qy, int qz, int lam, int trunc, int mode, int prior, int search, int n,
                      const int64_t *h, int64_t *out, int32_t *arg) {
    if (!check_args(1, 1, qx, qy, qz, lam, trunc, mode, prior, search) || n < 0) return OR_E_ARGS;
    prior_t p = make_prior(qx, qy, qz, lam, trunc, mode, prior);
    int64_t *scratch = malloc(sizeof(int64_t) * 8192);
    if (!scratch) return OR_E_NOMEM;
    for (int i = 0; i < n; ++i) {
        const int64_t *hi = h + (size_t)i * p.q;
        int64_t *oi = out + (size_t)i * p.q;
        if (search != 0) msearch(&p, search, hi, oi, scratch);
        else msearch_sfms(&p, hi, oi, arg ? arg + (size_t)i * p.q : NULL);
    }
    free(scratch);
    return OR_OK;
}

/* ---- EDP on a volume (D = 3) ---------------------------------------------- */

static int64_t floor_div3(int64_t s) { return s >= 0 ? s / 3 : -((-s + 2) / 3); }

/* Energy of eq. GE_objective_function on a 6-connected volume cost[Z][H][W][Q]. */
int64_t oracle_energy_volume(int W, int H, int Z, int qx, int qy, int lam, int trunc, int mode, int prior,
                             const int32_t *cost, const int32_t *labels) {
    prior_t p = make_prior(qx, qy, 1, lam, trunc, mode, prior);
    int64_t e = 0;
    for (int z = 0; z < Z; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t i = ((size_t)z * H + y) * W + x;
                int l = labels[i];
                e += cost[i * p.q + l];
                if (x + 1 < W) e += prior_v(&p, labels[i + 1], l);
                if (y + 1 < H) e += prior_v(&p, labels[i + W], l);
                if (z + 1 < Z) e += prior_v(&p, labels[i + (size_t)W * H], l);
            }
    return e;
}

/* direction k: 0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z; predecessor x_k = x - sgn(k) e_|k| */
static const int VDX[6] = {1, -1, 0, 0, 0, 0};
static const int VDY[6] = {0, 0, 1, -1, 0, 0};
static const int VDZ[6] = {0, 0, 0, 0, 1, -1};
static const int VOPP[6] = {1, 0, 3, 2, 5, 4};

/* Literal EDP on a volume: labels [Z][H][W]; marginal_out [Z][H][W][Q] int64 (nullable). */
int oracle_edp_volume(int W, int H, int Z, int qx, int qy, int lam, int trunc, int mode, int prior,
                      int iterations, int search, const int32_t *cost, int32_t *labels, int64_t *energy_out,
                      int64_t *max_abs_out, int64_t *marginal_out) {
    if (Z < 1 || !check_args(W, H, qx, qy, 1, lam, trunc, mode, prior, search) || iterations < 0) return OR_E_ARGS;
    prior_t p = make_prior(qx, qy, 1, lam, trunc, mode, prior);
    int Q = p.q;
    size_t cells = (size_t)W * H * Z;
    int64_t *S = calloc((size_t)6 * cells * Q, sizeof(int64_t));
    int64_t *h = malloc(sizeof(int64_t) * Q);
    int64_t *m = malloc(sizeof(int64_t) * 6 * Q);
    int64_t *acc = malloc(sizeof(int64_t) * Q);
    int64_t *scratch = malloc(sizeof(int64_t) * 8192);
    int64_t *nw = malloc(sizeof(int64_t) * 3 * Q);
    if (!S || !h || !m || !acc || !scratch || !nw) {
        free(S); free(h); free(m); free(acc); free(scratch); free(nw);
        return OR_E_NOMEM;
    }
    int64_t maxabs = 0;
    int status = OR_OK;
    for (int it = 0; it < iterations; ++it) {
        for (int scan = 0; scan < 8; ++scan) {
            const int sx = (scan & 1) ? -1 : 1, sy = (scan & 2) ? -1 : 1, sz = (scan & 4) ? -1 : 1;
            const int comp[3] = {sx > 0 ? 0 : 1, sy > 0 ? 2 : 3, sz > 0 ? 4 : 5};
            for (int zi = 0; zi < Z; ++zi) {
                int z = sz > 0 ? zi : Z - 1 - zi;
                for (int yi = 0; yi < H; ++yi) {
                    int y = sy > 0 ? yi : H - 1 - yi;
                    for (int xi = 0; xi < W; ++xi) {
                        int x = sx > 0 ? xi : W - 1 - xi;
                        for (int k = 0; k < 6; ++k) {   /* m_k = M(S_k(x_k) / 3), 0 off the grid */
                            int px = x - VDX[k], py = y - VDY[k], pz = z - VDZ[k];
                            int64_t *mk = m + (size_t)k * Q;
                            if (px < 0 || px >= W || py < 0 || py >= H || pz < 0 || pz >= Z) {
                                for (int v = 0; v < Q; ++v) mk[v] = 0;
                                continue;
                            }
                            const int64_t *sk = S + ((size_t)k * cells + ((size_t)pz * H + py) * W + px) * Q;
                            for (int v = 0; v < Q; ++v) h[v] = floor_div3(sk[v]);
                            msearch(&p, search, h, mk, scratch);
                        }
                        size_t cell = ((size_t)z * H + y) * W + x;
                        const int32_t *c = cost + cell * Q;
                        for (int j = 0; j < 3; ++j) {   /* eq. DP_2D_base with C added */
                            int kp = comp[j];
                            for (int v = 0; v < Q; ++v) {
                                int64_t s = c[v];
                                for (int k = 0; k < 6; ++k)
                                    if (k != VOPP[kp]) s += m[(size_t)k * Q + v];
                                s -= m[(size_t)VOPP[kp] * Q + v];
                                nw[(size_t)j * Q + v] = s;
                            }
                        }
                        for (int j = 0; j < 3; ++j) {
                            int64_t *dst = S + ((size_t)comp[j] * cells + cell) * Q;
                            for (int v = 0; v < Q; ++v) {
                                int64_t s = nw[(size_t)j * Q + v];
                                if (iabs64(s) > maxabs) maxabs = iabs64(s);
                                if (s > INT32_MAX || s < INT32_MIN) status = OR_E_RANGE;
                                dst[v] = s;
                            }
                        }
                    }
                }
            }
        }
    }
    for (int z = 0; z < Z; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {               /* eq. DP_2D_1 with C, eq. DP_2D_2 */
                size_t cell = ((size_t)z * H + y) * W + x;
                const int32_t *c = cost + cell * Q;
                for (int v = 0; v < Q; ++v) acc[v] = c[v];
                for (int k = 0; k < 6; ++k) {
                    int px = x - VDX[k], py = y - VDY[k], pz = z - VDZ[k];
                    if (px < 0 || px >= W || py < 0 || py >= H || pz < 0 || pz >= Z) continue;
                    const int64_t *sk = S + ((size_t)k * cells + ((size_t)pz * H + py) * W + px) * Q;
                    for (int v = 0; v < Q; ++v) h[v] = floor_div3(sk[v]);
                    msearch(&p, search, h, m, scratch);
                    for (int v = 0; v < Q; ++v) acc[v] += m[v];
                }
                int bi = 0;
                for (int v = 1; v < Q; ++v) if (acc[v] < acc[bi]) bi = v;
                labels[cell] = bi;
                if (marginal_out) memcpy(marginal_out + cell * Q, acc, sizeof(int64_t) * Q);
            }
    *energy_out = oracle_energy_volume(W, H, Z, qx, qy, lam, trunc, mode, prior, cost, labels);
    *max_abs_out = maxabs;
    free(S); free(h); free(m); free(acc); free(scratch); free(nw);
    return status;
}
