// Energy of a labelling (Mozerov, arXiv 1410.7922, Sec. 2 eq.
// GE_objective_function with the truncated linear or squared prior), data cost
// formation (Sec. 2 eq. Cost_value, Sec. 5.1 eq. Cost_cmp) and small helpers.
#include "edp_device.hpp"
#include "edp_internal.hpp"

namespace edp {

// V(u) of eq. Smooth_value_t with f(a) = |a| (squared false) or a^2 (squared true) between flat
// labels a and b = (vz qy + vy) qx + vx (qxy = qx qy; a two-dimensional space has vz = 0)
__device__ __forceinline__ int64_t prior_pair(int32_t a, int32_t b, int32_t qx, int32_t qxy, int32_t lam,
                                              int32_t trunc, bool joint, bool squared) {
    const int32_t ra = a % qxy, rb = b % qxy;
    int64_t dx = ra % qx - rb % qx, dy = ra / qx - rb / qx, dz = a / qxy - b / qxy;
    dx = dx < 0 ? -dx : dx;
    dy = dy < 0 ? -dy : dy;
    dz = dz < 0 ? -dz : dz;
    int64_t ft = trunc;
    if (squared) {
        dx *= dx;
        dy *= dy;
        dz *= dz;
        ft *= ft;
    }
    if (joint) return (int64_t)lam * (dx + dy + dz < ft ? dx + dy + dz : ft);
    return (int64_t)lam * ((dx < ft ? dx : ft) + (dy < ft ? dy : ft) + (dz < ft ? dz : ft));
}

template <class CT>
__global__ __launch_bounds__(256) void energy_kernel(const EnergyArgs a) {
    const int32_t W = a.W, H = a.H, QXY = a.qx * a.qy, Q = QXY * a.qz;
    const CT* __restrict__ cost = (const CT*)a.cost;
    const bool joint = a.joint != 0;
    int64_t acc = 0;
    unsigned long long bad = 0;
    const int64_t n = (int64_t)W * H;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int32_t y = (int32_t)(idx / W), x = (int32_t)(idx % W);
        const int32_t lab = a.labels[idx];
        if (lab < 0 || lab >= Q) { ++bad; continue; }
        acc += (int64_t)cost[idx * Q + lab];
        if (x + 1 < W) {
            const int32_t r = a.labels[idx + 1];
            if (r >= 0 && r < Q) acc += prior_pair(lab, r, a.qx, QXY, a.lam, a.trunc, joint, a.squared != 0);
        }
        if (a.grid4 && y + 1 < H) {
            const int32_t d = a.labels[idx + W];
            if (d >= 0 && d < Q) acc += prior_pair(lab, d, a.qx, QXY, a.lam, a.trunc, joint, a.squared != 0);
        }
    }
    __shared__ int64_t sacc[256];
    __shared__ unsigned long long sbad[256];
    sacc[threadIdx.x] = acc;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sacc[threadIdx.x] += sacc[threadIdx.x + st];
            sbad[threadIdx.x] += sbad[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // a solve whose scans gave up waiting reports INT64_MIN: no block adds, block 0 stores it
        if (a.error && *a.error != 0) {
            if (blockIdx.x == 0) *a.energy = (unsigned long long)INT64_MIN;
        } else {
            atomicAdd(a.energy, (unsigned long long)sacc[0]);
        }
        if (a.invalid) atomicAdd(a.invalid, sbad[0]);
    }
}

// Energies of a batch class: block b covers rows_per_block rows of the instance
// that holds it and adds its share to that instance's energy word.  The scans ran before this
// launch on the same stream, so their error word is final: if it is set, the first block of each
// instance stores INT64_MIN and no block adds.  With a.status the first block also writes the
// instance's status word (classes whose last scan formed the labels).
template <class CT>
__global__ __launch_bounds__(256) void batch_energy_kernel(const BatchEnergyArgs a) {
    const InstDesc d = uniform_desc(a.descs[find_instance(a.descs, a.ndesc, (int32_t)blockIdx.x, 2)]);
    const bool failed = a.error && *a.error != 0;
    const bool first = (int32_t)blockIdx.x == d.first_eblock;
    if (threadIdx.x == 0 && first) {
        if (a.status && d.status) *d.status = failed ? STATUS_TIMEOUT : 0;
        if (failed && d.energy) *d.energy = (unsigned long long)INT64_MIN;
    }
    if (failed) return;
    const int32_t W = d.W, H = d.H, QXY = d.qx * d.qy, Q = QXY * d.qz;
    const CT* __restrict__ cost = (const CT*)d.cost;
    const bool joint = d.joint != 0;
    const int32_t y0 = ((int32_t)blockIdx.x - d.first_eblock) * a.rows_per_block;
    const int32_t y1 = y0 + a.rows_per_block < H ? y0 + a.rows_per_block : H;
    int64_t acc = 0;
    for (int32_t y = y0; y < y1; ++y) {
        for (int32_t x = threadIdx.x; x < W; x += blockDim.x) {
            const int64_t idx = (int64_t)y * W + x;
            const int32_t lab = d.labels[idx];
            if (lab < 0 || lab >= Q) continue;
            acc += (int64_t)cost[idx * Q + lab];
            if (x + 1 < W) {
                const int32_t r = d.labels[idx + 1];
                if (r >= 0 && r < Q) acc += prior_pair(lab, r, d.qx, QXY, d.lam, d.trunc, joint, d.squared != 0);
            }
            if (y + 1 < H) {
                const int32_t v = d.labels[idx + W];
                if (v >= 0 && v < Q) acc += prior_pair(lab, v, d.qx, QXY, d.lam, d.trunc, joint, d.squared != 0);
            }
        }
    }
    __shared__ int64_t sacc[256];
    sacc[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sacc[threadIdx.x] += sacc[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0 && d.energy) atomicAdd(d.energy, (unsigned long long)sacc[0]);
}

// p[0 .. n) = v; the words from the first 16-byte boundary on go out four at a time
// p[0, n) = v (16-byte stores), and the few words p2[0, n2) = v as well (block 0)
__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v, uint32_t* p2, uint32_t n2) {
    if (blockIdx.x == 0 && threadIdx.x < n2) p2[threadIdx.x] = v;
    const size_t head = ((16 - ((uintptr_t)p & 15)) & 15) / 4;
    const size_t h = head < n ? head : n;
    const size_t nv = (n - h) / 4;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, step = (size_t)gridDim.x * blockDim.x;
    if (tid < h) p[tid] = v;
    uint4* q = (uint4*)(p + h);
    const uint4 w = make_uint4(v, v, v, v);
    for (size_t i = tid; i < nv; i += step) q[i] = w;
    for (size_t i = h + 4 * nv + tid; i < n; i += step) p[i] = v;
}

__global__ __launch_bounds__(256) void sum_rows_kernel(const int64_t* rows, int32_t n, int64_t* out) {
    __shared__ int64_t s[256];
    int64_t acc = 0;
    for (int32_t i = threadIdx.x; i < n; i += 256) acc += rows[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

__global__ void copy_i64_kernel(const int64_t* src, int64_t* dst, int32_t n) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

hipError_t launch_energy(int dtype, const EnergyArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)a.W * a.H;
    int grid = (int)((n + 255) / 256);
    if (grid > 2048) grid = 2048;
    if (grid < 1) grid = 1;
    if (dtype == 1)
        hipLaunchKernelGGL(energy_kernel<int16_t>, dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(energy_kernel<int32_t>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Label-window solve, preparation: cw[cell][jy * 8 + jx] = C(cell, window label (jx, jy)) for
// jx, jy < win, big elsewhere in the 8 x 8 frame; shifts[cell] = frame offsets (dx, dy) of the
// four neighbours' windows relative to this vertex's (int8 pairs: +x, -x | +y, -y; 0 off grid).
__global__ __launch_bounds__(256) void win_prep_kernel(const int32_t* cost, const int32_t* centers, int32_t W,
                                                       int32_t H, int32_t qx, int32_t qy, int32_t win, int32_t big,
                                                       int32_t* cw, uint32_t* shifts) {
    const int64_t total = (int64_t)W * H * WIN_FRAME * WIN_FRAME;
    const int32_t Q = qx * qy, r = win / 2;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cell = idx / (WIN_FRAME * WIN_FRAME);
        const int32_t slot = (int32_t)(idx % (WIN_FRAME * WIN_FRAME));
        const int32_t jx = slot % WIN_FRAME, jy = slot / WIN_FRAME;
        const int32_t cx = centers[2 * cell], cy = centers[2 * cell + 1];
        const int32_t vx = cx - r + jx, vy = cy - r + jy;
        const bool in = jx < win && jy < win && vx >= 0 && vx < qx && vy >= 0 && vy < qy;
        cw[idx] = in ? cost[cell * Q + vy * qx + vx] : big;
        if (slot == 0) {
            const int32_t x = (int32_t)(cell % W), y = (int32_t)(cell / W);
            const int32_t nx[4] = {x + 1, x - 1, x, x}, ny[4] = {y, y, y + 1, y - 1};
            uint32_t code[2] = {0u, 0u};
            for (int k = 0; k < 4; ++k) {
                int32_t ddx = 0, ddy = 0;
                if (nx[k] >= 0 && nx[k] < W && ny[k] >= 0 && ny[k] < H) {
                    const int64_t n = (int64_t)ny[k] * W + nx[k];
                    ddx = centers[2 * n] - cx;
                    ddy = centers[2 * n + 1] - cy;
                }
                const uint32_t pair = ((uint32_t)ddx & 0xFFu) | (((uint32_t)ddy & 0xFFu) << 8);
                code[k >> 1] |= pair << (16 * (k & 1));
            }
            shifts[2 * cell] = code[0];
            shifts[2 * cell + 1] = code[1];
        }
    }
}

hipError_t launch_win_prep(const int32_t* cost, const int32_t* centers, int32_t W, int32_t H, int32_t qx, int32_t qy,
                           int32_t win, int32_t big, int32_t* cw, uint32_t* shifts, hipStream_t s) {
    const int64_t n = (int64_t)W * H * WIN_FRAME * WIN_FRAME;
    int64_t grid = (n + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(win_prep_kernel, dim3((unsigned)grid), dim3(256), 0, s, cost, centers, W, H, qx, qy, win, big,
                       cw, shifts);
    return hipGetLastError();
}

hipError_t launch_batch_energy(int dtype, const BatchEnergyArgs& a, int grid, hipStream_t s) {
    if (grid < 1) return hipSuccess;
    if (dtype == 1)
        hipLaunchKernelGGL(batch_energy_kernel<int16_t>, dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(batch_energy_kernel<int32_t>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---- data cost (DSI) formation -------------------------------------------------------------
// Sec. 2 eq. Cost_value, min(|I1(x + v) - I0(x)|^l2, cmax), and with a third image the composite
// cost of Sec. 5.1 eq. Cost_cmp, min(C_{0->1}(x, v), C_{0->2}(x, -v)).  Each thread forms V
// consecutive elements of the [H][W][Q] volume (16 bytes) and stores them with one vector store.
// The kernel is bound by its per-element instructions: the displacements of all labels sit in an
// LDS table (dx, dy as two 16-bit halves), so an element costs a table read, the displaced
// position and its bounds, two byte loads and the truncated difference; the step to the next
// label, pixel and row is made of selects, so the code is straight-line and the loads of all V
// elements are in flight together.  An out-of-image position uses the out-of-range buffer offset (the load
// returns 0) and the element takes cmax.
template <int L2>
__device__ __forceinline__ int32_t dsi_view(__amdgpu_buffer_rsrc_t img, int32_t c0, int32_t x, int32_t y,
                                            int32_t W, int32_t H, int32_t cmax) {
    const bool ok = (uint32_t)x < (uint32_t)W && (uint32_t)y < (uint32_t)H;
    int32_t d = (int32_t)__builtin_amdgcn_raw_buffer_load_b8(img, ok ? y * W + x : OOB, 0, 0) - c0;
    d = d < 0 ? -d : d;
    if constexpr (L2 == 2) d *= d;
    d = d < cmax ? d : cmax;
    // the truncated cost is at most cmax: raising it to cmax off the image takes no select on the
    // loaded value, so the load is not moved under a branch
    const int32_t floor_v = ok ? 0 : cmax;
    return d > floor_v ? d : floor_v;
}

template <class CT, int L2, bool COMP>
__global__ __launch_bounds__(256) void dsi_kernel(const DsiArgs a) {
    constexpr int V = 16 / (int)sizeof(CT);
    extern __shared__ int32_t disp[];                  // [Q] (dx & 0xFFFF) | (dy << 16)
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy;
    for (int32_t i = threadIdx.x; i < Q; i += blockDim.x) {
        const int32_t iy = i / a.qx, ix = i - iy * a.qx;
        const int32_t dx = a.ox + a.sx * ix, dy = a.oy + a.sy * iy;
        disp[i] = (int32_t)(((uint32_t)dx & 0xFFFFu) | ((uint32_t)dy << 16));
    }
    __syncthreads();
    const int64_t n = (int64_t)W * H * Q;
    const __amdgpu_buffer_rsrc_t r0 = make_rsrc(a.i0, W * H);
    const __amdgpu_buffer_rsrc_t r1 = make_rsrc(a.i1, W * H);
    const __amdgpu_buffer_rsrc_t r2 = make_rsrc(a.i2, COMP ? W * H : 0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * V;
    for (int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * V; base < n; base += stride) {
        // base / Q and pix / W through double reciprocals: (e + 1/2) / d is at least 1/(2d) away
        // from an integer and the product's error is far below that for e < 2^50, so the floor is
        // exact (a 64-bit integer division costs more than the 16 bytes it indexes)
        const int64_t pix = (int64_t)(((double)base + 0.5) * a.inv_q);
        int32_t q = (int32_t)(base - pix * Q);
        int32_t y = (int32_t)(((double)pix + 0.5) * a.inv_w), x = (int32_t)(pix - (int64_t)y * W);
        CT out[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            // every element loads its own I0 byte (a cache hit)
            const int32_t c0 = (int32_t)__builtin_amdgcn_raw_buffer_load_b8(r0, y < H ? y * W + x : OOB, 0, 0);
            const int32_t t = disp[q];
            const int32_t dx = (int32_t)(int16_t)(t & 0xFFFF), dy = t >> 16;
            int32_t c = dsi_view<L2>(r1, c0, x + dx, y + dy, W, H, a.cmax);
            if constexpr (COMP) {
                const int32_t c2 = dsi_view<L2>(r2, c0, x - dx, y - dy, W, H, a.cmax);
                c = c < c2 ? c : c2;
            }
            out[k] = (CT)c;
            // next element, with selects only: straight-line code lets every load go out first
            const bool next_pixel = ++q == Q;
            q = next_pixel ? 0 : q;
            x += next_pixel ? 1 : 0;
            const bool next_row = x == W;
            x = next_row ? 0 : x;
            y += next_row ? 1 : 0;
        }
        CT* dst = (CT*)a.cost + base;
        if (a.vec && base + V <= n) {
            uint4 w;
            __builtin_memcpy(&w, out, 16);
            *(uint4*)dst = w;
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (base + k < n) dst[k] = out[k];
        }
    }
}

// Staged windows: one workgroup forms the costs of a segment of up to seg pixels of one row.
// All I1 values those pixels compare with (qy rows of pw = seg + qx - 1 pixels), and the I2
// values of the composite cost, are read once into LDS as 16-bit values, 0xFFFF off the image;
// a table gives each label's offset into the windows (I2's in the upper half), so an element
// costs the table read, one or two window reads, the I0 value of its pixel and the truncated
// difference, with no global gathers.  The segment's elements are a contiguous run of the
// volume: whole 16-byte vectors in the middle, single elements at both ends.
template <int L2>
__device__ __forceinline__ int32_t window_cost(uint32_t v, int32_t c0, int32_t cmax) {
    int32_t d = (int32_t)(v & 0xFFu) - c0;
    d = d < 0 ? -d : d;
    if constexpr (L2 == 2) d *= d;
    d = d < cmax ? d : cmax;
    return v > 255u ? cmax : d;
}

template <class CT, int L2, bool COMP>
__global__ __launch_bounds__(256) void dsi_window_kernel(const DsiArgs a) {
    constexpr int V = 16 / (int)sizeof(CT);
    extern __shared__ int32_t smem[];
    const int32_t W = a.W, H = a.H, Q = a.qx * a.qy, PW = a.pw, NE = a.qy * a.pw;
    // [Q] window offsets, label q at q + q / 4: the 4 consecutive labels of a lane's vector sit
    // 5 words from the next lane's, so the lanes of a wavefront read 32 different banks
    int32_t* const tab = smem;
    uint16_t* const w1 = (uint16_t*)(smem + Q + (Q >> 2) + 1);   // [qy][pw] I1
    uint16_t* const w2 = w1 + NE;                                // [qy][pw] I2 (COMP)
    uint16_t* const row0 = w2 + (COMP ? NE : 0);                 // [seg] I0 of the segment
    const int32_t y = blockIdx.x / a.nseg, x0 = (blockIdx.x - y * a.nseg) * a.seg;
    const int32_t np = W - x0 < a.seg ? W - x0 : a.seg;
    for (int32_t i = threadIdx.x; i < Q; i += blockDim.x) {
        const int32_t iy = i / a.qx, ix = i - iy * a.qx;
        const int32_t dx = a.ox + a.sx * ix, dy = a.oy + a.sy * iy;
        const int32_t o1 = (dy - a.dymin) * PW + (dx - a.dxmin);
        const int32_t o2 = COMP ? (a.dymax - dy) * PW + (a.dxmax - dx) : 0;
        tab[i + (i >> 2)] = o1 | (o2 << 16);
    }
    // pixel x0 + p at displacement (dx, dy) reads w1[o1 + p] = I1(x0 + p + dx, y + dy) and
    // w2[o2 + p] = I2(x0 + p - dx, y - dy)
    for (int32_t i = threadIdx.x; i < NE; i += blockDim.x) {
        const int32_t r = i / PW, c = i - r * PW;
        const int32_t X1 = x0 + a.dxmin + c, Y1 = y + a.dymin + r;
        const bool ok1 = (uint32_t)X1 < (uint32_t)W && (uint32_t)Y1 < (uint32_t)H;
        w1[i] = ok1 ? (uint16_t)a.i1[(size_t)Y1 * W + X1] : (uint16_t)0xFFFF;
        if constexpr (COMP) {
            const int32_t X2 = x0 - a.dxmax + c, Y2 = y - a.dymax + r;
            const bool ok2 = (uint32_t)X2 < (uint32_t)W && (uint32_t)Y2 < (uint32_t)H;
            w2[i] = ok2 ? (uint16_t)a.i2[(size_t)Y2 * W + X2] : (uint16_t)0xFFFF;
        }
    }
    for (int32_t i = threadIdx.x; i < np; i += blockDim.x) row0[i] = a.i0[(size_t)y * W + x0 + i];
    __syncthreads();

    auto elem = [&](int32_t p, int32_t q) -> int32_t {
        const uint32_t t = (uint32_t)tab[q + (q >> 2)];
        const int32_t c0 = row0[p];
        int32_t c = window_cost<L2>(w1[(t & 0xFFFFu) + p], c0, a.cmax);
        if constexpr (COMP) {
            const int32_t c2 = window_cost<L2>(w2[(t >> 16) + p], c0, a.cmax);
            c = c < c2 ? c : c2;
        }
        return c;
    };
    CT* const cost = (CT*)a.cost;
    const int64_t E0 = ((int64_t)y * W + x0) * Q, E1 = E0 + (int64_t)np * Q;
    int64_t A0 = (E0 + V - 1) / V * V, A1 = E1 / V * V;
    if (A0 > A1) A0 = A1 = E1;
    // single elements before the first and after the last whole vector
    for (int64_t e = E0 + threadIdx.x; e < A0; e += blockDim.x) {
        const int32_t l = (int32_t)(e - E0), p = l / Q;
        cost[e] = (CT)elem(p, l - p * Q);
    }
    for (int64_t e = A1 + threadIdx.x; e < E1; e += blockDim.x) {
        const int32_t l = (int32_t)(e - E0), p = l / Q;
        cost[e] = (CT)elem(p, l - p * Q);
    }
    for (int64_t e = A0 + (int64_t)threadIdx.x * V; e < A1; e += (int64_t)blockDim.x * V) {
        // l < seg * Q <= 2^18: the float quotient of l + 1/2 is at least 1/(2Q) from an
        // integer and its error is below 2^-16, so the floor is exact
        const int32_t l = (int32_t)(e - E0);
        int32_t p = (int32_t)(((float)l + 0.5f) * a.inv_qf);
        int32_t q = l - p * Q;
        CT out[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            out[k] = (CT)elem(p, q);
            const bool next_pixel = ++q == Q;
            q = next_pixel ? 0 : q;
            p += next_pixel ? 1 : 0;
        }
        uint4 w;
        __builtin_memcpy(&w, out, 16);
        *(uint4*)(cost + e) = w;
    }
}

// LDS of the staged-window kernel (bytes)
static size_t dsi_window_lds(int32_t qx, int32_t qy, int32_t seg, bool comp) {
    const size_t ne = (size_t)qy * (size_t)(seg + qx - 1);
    const size_t q = (size_t)qx * qy;
    return (q + q / 4 + 1) * 4 + (comp ? 2 : 1) * ne * 2 + (size_t)seg * 2 + 4;
}

template <class CT>
static void run_dsi_window(const DsiArgs& a, hipStream_t s) {
    const size_t lds = dsi_window_lds(a.qx, a.qy, a.seg, a.i2 != nullptr);
    const int grid = a.H * a.nseg;
    if (a.l2 == 2) {
        if (a.i2) hipLaunchKernelGGL((dsi_window_kernel<CT, 2, true>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((dsi_window_kernel<CT, 2, false>), dim3(grid), dim3(256), lds, s, a);
    } else {
        if (a.i2) hipLaunchKernelGGL((dsi_window_kernel<CT, 1, true>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((dsi_window_kernel<CT, 1, false>), dim3(grid), dim3(256), lds, s, a);
    }
}

template <class CT>
static void run_dsi(const DsiArgs& a, int grid, hipStream_t s) {
    const size_t lds = (size_t)a.qx * a.qy * 4;
    if (a.l2 == 2) {
        if (a.i2) hipLaunchKernelGGL((dsi_kernel<CT, 2, true>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((dsi_kernel<CT, 2, false>), dim3(grid), dim3(256), lds, s, a);
    } else {
        if (a.i2) hipLaunchKernelGGL((dsi_kernel<CT, 1, true>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((dsi_kernel<CT, 1, false>), dim3(grid), dim3(256), lds, s, a);
    }
}

hipError_t launch_dsi(const DsiArgs& args, int dtype, hipStream_t s) {
    DsiArgs a = args;
    const int V = dtype == 1 ? 8 : 4;
    const int32_t Q = a.qx * a.qy, esize = dtype == 1 ? 2 : 4;
    // staged windows when the output takes vector stores and the windows fit 64 KB of LDS:
    // 64-pixel segments, 256 when a pixel's labels fill less than 512 bytes
    const bool comp = a.i2 != nullptr;
    int32_t seg = Q * esize < 512 ? 256 : 64;
    if (dsi_window_lds(a.qx, a.qy, seg, comp) > 65536) seg = 64;
    if (a.vec && dsi_window_lds(a.qx, a.qy, seg, comp) <= 65536) {
        a.seg = seg;
        a.nseg = (a.W + seg - 1) / seg;
        a.pw = seg + a.qx - 1;
        const int32_t dx1 = a.ox + a.sx * (a.qx - 1), dy1 = a.oy + a.sy * (a.qy - 1);
        a.dxmin = a.ox < dx1 ? a.ox : dx1;
        a.dxmax = a.ox < dx1 ? dx1 : a.ox;
        a.dymin = a.oy < dy1 ? a.oy : dy1;
        a.dymax = a.oy < dy1 ? dy1 : a.oy;
        a.inv_qf = 1.0f / (float)Q;
        if (dtype == 1) run_dsi_window<int16_t>(a, s);
        else run_dsi_window<int32_t>(a, s);
        return hipGetLastError();
    }
    const int64_t n = (int64_t)a.W * a.H * a.qx * a.qy;
    int64_t grid = (n / V + 255) / 256 + 1;
    if (grid > 65536) grid = 65536;
    if (dtype == 1) run_dsi<int16_t>(a, (int)grid, s);
    else run_dsi<int32_t>(a, (int)grid, s);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    return launch_fill_u32_with(p, n, nullptr, 0, v, s);
}

hipError_t launch_fill_u32_with(uint32_t* p, size_t n, uint32_t* p2, uint32_t n2, uint32_t v, hipStream_t s) {
    if (n == 0 && n2 == 0) return hipSuccess;
    size_t grid = (n / 4 + 255) / 256 + 1;
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)grid), dim3(256), 0, s, p, n, v, p2, n2);
    return hipGetLastError();
}

hipError_t launch_sum_rows(const int64_t* rows, int32_t n, int64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(256), 0, s, rows, n, out);
    return hipGetLastError();
}

hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, int32_t n, hipStream_t s) {
    int grid = (n + 255) / 256;
    if (grid > 256) grid = 256;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(copy_i64_kernel, dim3(grid), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace edp
