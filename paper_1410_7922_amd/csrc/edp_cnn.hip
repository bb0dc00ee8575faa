// Label-window network kernels for gfx950: motion cost volume (Sec. 2
// eq. Cost_value with the squared difference), pooled network input, 3x3
// convolutions as implicit GEMMs on bf16 matrix cores (v_mfma_f32_16x16x32_bf16,
// float accumulation) for the forward pass, the input gradient and the weight
// gradient, softmax cross entropy, Adam, and the decoding of the logits into
// per-pixel label windows.
//
// Layouts: activations channels-last [h][w][C] bf16 (uint16 storage); weights
// [Cout][3][3][Cin] bf16; the logits / gradients float32 [h][w][ld].
#include <stdint.h>

#include "edp_internal.hpp"

namespace edp {

// The network's kernels and helpers (a named namespace, so traces show the kernel names).
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// float -> bf16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ u32x4 load16(const uint16_t* p) { return *(const u32x4*)p; }

// ---------------------------------------------------------------------------
// cost volume and network input
// ---------------------------------------------------------------------------

// C(x, y, q) = min((I0(x, y) - I1(x + dx, y + dy))^2, cmax), q = (dy + r)(2r + 1) + (dx + r);
// a displaced pixel outside the frame costs cmax.
__global__ void dsi_motion_kernel(const uint8_t* i0, const uint8_t* i1, int32_t W, int32_t H, int32_t r,
                                  int32_t cmax, int32_t* out) {
    const int32_t n = 2 * r + 1, nn = n * n;
    const int64_t total = (int64_t)W * H * nn;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = (int32_t)(idx % nn);
        const int64_t pix = idx / nn;
        const int32_t x = (int32_t)(pix % W), y = (int32_t)(pix / W);
        const int32_t x2 = x + q % n - r, y2 = y + q / n - r;
        int32_t c = cmax;
        if (x2 >= 0 && x2 < W && y2 >= 0 && y2 < H) {
            const int32_t d = (int32_t)i0[pix] - (int32_t)i1[(int64_t)y2 * W + x2];
            c = d * d < cmax ? d * d : cmax;
        }
        out[idx] = c;
    }
}

// Network input.  One wavefront per half-resolution pixel.  The label blocks of its 2 x 2
// pixels (Q <= 1024 int32 each) are read with coalesced dword loads -- lane l takes labels l,
// l + 64, ..., all loads of the four pixels in flight together -- into the wavefront's LDS area
// [4][Q]; then lane c takes channel c.  mode 0: channel = block of 4 x 4 labels (bx * by <= 64),
// the minimum over the block; mode 1: channel c < qx is the minimum over the label column c,
// channel qx + r the minimum over the label row r (qx + qy <= 64), further channels 0.  Each
// minimum is summed over the 2 x 2 pixels and divided by 4 scale (one float32 division).
constexpr int POOL_QMAX = 1024;
__global__ __launch_bounds__(256) void pool_kernel(const int32_t* cost, int32_t W, int32_t H, int32_t qx,
                                                   int32_t qy, int32_t scale, int32_t nbx, int32_t nch,
                                                   int32_t mode, uint16_t* out) {
    extern __shared__ int32_t pool_lds[];          // [4 wavefronts][4 pixels][Q]
    constexpr int NL = POOL_QMAX / 64;             // loads per lane and pixel at most
    const int32_t w2 = W / 2, h2 = H / 2;
    const int32_t wave = (int32_t)(threadIdx.x >> 6), lane = (int32_t)(threadIdx.x & 63);
    const int64_t opix = (int64_t)blockIdx.x * 4 + wave;
    if (opix >= (int64_t)w2 * h2) return;          // the whole wavefront leaves; no workgroup barrier follows
    const int32_t X = (int32_t)(opix % w2), Y = (int32_t)(opix / w2);
    const int32_t Q = qx * qy;
    int32_t* buf = pool_lds + (size_t)wave * 4 * Q;
    int32_t v[4][NL];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t* c = cost + ((int64_t)(2 * Y + (k >> 1)) * W + (2 * X + (k & 1))) * Q;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int32_t i = lane + 64 * j;
            v[k][j] = i < Q ? __builtin_nontemporal_load(c + i) : 0;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int32_t i = lane + 64 * j;
            if (i < Q) buf[k * Q + i] = v[k][j];
        }
    // the wavefront's LDS writes are performed before its reads below (LDS executes a wavefront's
    // operations in order); the fence keeps the compiler from moving the reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane >= nch) return;
    int32_t x0, x1, y0, y1;
    if (mode == 0) {
        const int32_t bxi = lane % nbx, byi = lane / nbx;
        x0 = bxi * 4;
        x1 = x0 + 4 < qx ? x0 + 4 : qx;
        y0 = byi * 4;
        y1 = y0 + 4 < qy ? y0 + 4 : qy;
    } else if (lane < qx) {
        x0 = lane, x1 = lane + 1, y0 = 0, y1 = qy;
    } else if (lane < qx + qy) {
        x0 = 0, x1 = qx, y0 = lane - qx, y1 = lane - qx + 1;
    } else {
        out[opix * nch + lane] = 0;
        return;
    }
    int64_t sum = 0;
    for (int k = 0; k < 4; ++k) {
        const int32_t* c = buf + k * Q;
        int32_t m = 0x7FFFFFFF;
        for (int32_t vy = y0; vy < y1; ++vy)
            for (int32_t vx = x0; vx < x1; ++vx) m = min(m, c[vy * qx + vx]);
        sum += m;
    }
    out[opix * nch + lane] = f2bf((float)sum / (float)(4 * scale));
}

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit GEMM on the matrix cores
// ---------------------------------------------------------------------------
//
// v_mfma_f32_16x16x32_bf16: A is 16 x 32 (lane l holds row l % 16, k = 8 (l / 16) .. + 7),
// B is 32 x 16 (lane l holds column l % 16, the same k range), D is 16 x 16 float (lane l
// holds column l % 16, rows 4 (l / 16) .. + 3).  Rows are pixels, columns output channels,
// k runs over (tap, input channel).

// out[p][co] = sum_{tap, ci} in[p + off(tap)][ci] * w[co][tap][ci] (+ bias, ReLU), or the
// input gradient with the flipped weights (then mask by the layer input being positive).
// One wavefront computes 16 pixels x all COUT; a workgroup covers 64 pixels.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias, int32_t h, int32_t wd,
                                                   int32_t cout_real, int32_t relu, int32_t dil,
                                                   const uint16_t* __restrict__ mask_in, int32_t ld_out,
                                                   uint16_t* __restrict__ out_bf, float* __restrict__ out_f) {
    constexpr int NT = COUT / 16;
    const int32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)h * wd;
    const int64_t p0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int64_t pa = p0 + (lane & 15);            // this lane's A row (pixel)
    const int32_t ya = (int32_t)(pa / wd), xa = (int32_t)(pa % wd);
    const int32_t kq = 8 * (lane >> 4);             // this lane's k offset within a 32-wide step
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
        const int32_t ys = ya + (tap / 3 - 1) * dil, xs = xa + (tap % 3 - 1) * dil;
        const bool ok = pa < P && ys >= 0 && ys < h && xs >= 0 && xs < wd;
        const uint16_t* src = in + ((int64_t)ys * wd + xs) * CIN + kq;
#pragma unroll
        for (int cb = 0; cb < CIN; cb += 32) {
            const u32x4 av = ok ? load16(src + cb) : u32x4{0u, 0u, 0u, 0u};
            const bf16x8 a = __builtin_bit_cast(bf16x8, av);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int32_t co = t * 16 + (lane & 15);
                const u32x4 bv = co < cout_real ? load16(w + ((int64_t)co * 9 + tap) * CIN + cb + kq)
                                                : u32x4{0u, 0u, 0u, 0u};
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int32_t co = t * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t p = p0 + 4 * (lane >> 4) + i;
            if (p >= P) continue;
            float v = acc[t][i];
            if (co >= cout_real) v = 0.f;
            else {
                if (bias) v += bias[co];
                if (relu) v = v > 0.f ? v : 0.f;
                if (mask_in && !(bf2f(mask_in[p * COUT + co]) > 0.f)) v = 0.f;
            }
            if (out_f) out_f[p * ld_out + co] = v;
            if (out_bf) out_bf[p * ld_out + co] = f2bf(v);
        }
    }
}

// wt[ci][tap][co] = w[co][8 - tap][ci] for co < cout (zero for the padded co)
__global__ void flip_kernel(const uint16_t* w, int32_t cin, int32_t cout, int32_t cout_pad, uint16_t* wt) {
    const int32_t n = cin * 9 * cout_pad;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t co = i % cout_pad, tap = (i / cout_pad) % 9, ci = i / (cout_pad * 9);
        wt[i] = co < cout ? w[((int64_t)co * 9 + (8 - tap)) * cin + ci] : (uint16_t)0;
    }
}

// dw[co][tap][ci] += sum_p dy[p][co] * x[p + off(tap)][ci].  Workgroup (tap, pixel stripe):
// chunks of 32 pixels are staged transposed in LDS, so both operands read 16 contiguous bytes.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t* __restrict__ dy, const uint16_t* __restrict__ x,
                                                    int32_t h, int32_t wd, int32_t cout_real, int32_t dil,
                                                    float* __restrict__ dw) {
    constexpr int KS = 40;                          // LDS row stride (elements), 16-byte multiple
    constexpr int MT = COUT / 16, NTL = CIN / 16, TILES = MT * NTL;
    constexpr int PER = (TILES + 3) / 4;
    __shared__ __align__(16) uint16_t dyt[COUT * KS];
    __shared__ __align__(16) uint16_t xt[CIN * KS];
    const int32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t tap = blockIdx.x;
    const int32_t dyo = (tap / 3 - 1) * dil, dxo = (tap % 3 - 1) * dil;
    const int64_t P = (int64_t)h * wd;
    const int64_t nchunk = (P + 31) / 32;
    f32x4 acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t c = blockIdx.y; c < nchunk; c += gridDim.y) {
        const int64_t pbase = c * 32;
        // stage: dyt[co][k] = dy[pbase + k][co], xt[ci][k] = x[pbase + k + off][ci]
        for (int32_t e = threadIdx.x; e < 32 * COUT; e += 256) {
            const int32_t k = e / COUT, co = e % COUT;
            const int64_t p = pbase + k;
            dyt[co * KS + k] = p < P ? dy[p * COUT + co] : (uint16_t)0;
        }
        for (int32_t e = threadIdx.x; e < 32 * CIN; e += 256) {
            const int32_t k = e / CIN, ci = e % CIN;
            const int64_t p = pbase + k;
            uint16_t v = 0;
            if (p < P) {
                const int32_t yy = (int32_t)(p / wd) + dyo, xx = (int32_t)(p % wd) + dxo;
                if (yy >= 0 && yy < h && xx >= 0 && xx < wd) v = x[((int64_t)yy * wd + xx) * CIN + ci];
            }
            xt[ci * KS + k] = v;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int tile = wave + 4 * i;
            if (tile < TILES) {
                const int mt = tile / NTL, nt = tile % NTL;
                const u32x4 av = *(const u32x4*)&dyt[(mt * 16 + (lane & 15)) * KS + 8 * (lane >> 4)];
                const u32x4 bv = *(const u32x4*)&xt[(nt * 16 + (lane & 15)) * KS + 8 * (lane >> 4)];
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                  __builtin_bit_cast(bf16x8, bv), acc[i], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int tile = wave + 4 * i;
        if (tile >= TILES) continue;
        const int mt = tile / NTL, nt = tile % NTL;
        const int32_t ci = nt * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int32_t co = mt * 16 + 4 * (lane >> 4) + r;
            if (co < cout_real) atomicAdd(&dw[((int64_t)co * 9 + tap) * CIN + ci], acc[i][r]);
        }
    }
}

// out[c] += sum over rows of a[r][c] (c < cols)
__global__ __launch_bounds__(256) void colsum_kernel(const float* a, int32_t rows, int32_t cols, int32_t ld,
                                                     float* out) {
    const int32_t c = threadIdx.x & 63;
    const int32_t g = blockIdx.x * 4 + (threadIdx.x >> 6), ng = gridDim.x * 4;
    if (c >= cols) return;
    float s = 0.f;
    for (int32_t r = g; r < rows; r += ng) s += a[(int64_t)r * ld + c];
    atomicAdd(&out[c], s);
}

// Per pixel and head, the negative log softmax mass of the window of win labels (clamped into
// [0, nclass)) around the target, averaged over the n pixels and summed over the heads; win = 1
// is the softmax cross entropy.  d/dz_k = (p_k - [k in window] p_k / mass) / n.
__global__ __launch_bounds__(256) void ce_kernel(const float* logits, int32_t n, int32_t ld, const int32_t* tx,
                                                 const int32_t* ty, int32_t nclass, int32_t win, float* grad_f,
                                                 uint16_t* grad_bf, float* loss) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (p < n) {
        const float* z = logits + (int64_t)p * ld;
        const int32_t r = win / 2;
        for (int head = 0; head < 2; ++head) {
            const int32_t t = head == 0 ? tx[p] : ty[p];
            const int32_t c = min(max(t, r), nclass - 1 - r);
            const float* zh = z + head * nclass;
            float m = zh[0];
            for (int k = 1; k < nclass; ++k) m = fmaxf(m, zh[k]);
            float s = 0.f, sw = 0.f;
            for (int k = 0; k < nclass; ++k) {
                const float e = expf(zh[k] - m);
                s += e;
                if (k >= c - r && k <= c + r) sw += e;
            }
            l += logf(s) - logf(sw);
            const float inv = 1.f / s, invw = 1.f / sw;
            for (int k = 0; k < nclass; ++k) {
                const float e = expf(zh[k] - m);
                float g = e * inv;
                if (k >= c - r && k <= c + r) g -= e * invw;
                g /= (float)n;
                const int64_t o = (int64_t)p * ld + head * nclass + k;
                grad_f[o] = g;
                grad_bf[o] = f2bf(g);
            }
        }
        for (int k = 2 * nclass; k < ld; ++k) {
            grad_f[(int64_t)p * ld + k] = 0.f;
            grad_bf[(int64_t)p * ld + k] = 0;
        }
    }
    // block sum of the per-pixel losses, one atomic per block
    __shared__ float red[256];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] / (float)n);
}

// Adam with each gradient element clipped to [-clip, clip] (clip > 0) and non-finite elements
// dropped, so one bad step cannot poison the moments.
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, uint16_t* pb, int32_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2, float clip) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float gi = g[i];
        if (!(fabsf(gi) <= 3.0e38f)) gi = 0.f;
        if (clip > 0.f) gi = fminf(fmaxf(gi, -clip), clip);
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        pb[i] = f2bf(pi);
    }
}

// Per half-resolution pixel and head: the window of largest probability mass.  With
// m_c = sum_{|k-c| <= win/2} exp(z_k - max z) for c in [win/2, q-1-win/2], the centre is the
// first c with m_c >= (1 - 1e-5) max m (near-equal windows resolve to the lowest centre),
// written to the 2 x 2 full-resolution pixels it covers.
__global__ void decode_kernel(const float* logits, int32_t h, int32_t w, int32_t ld, int32_t qx, int32_t qy,
                              int32_t win, int32_t nclass, int32_t* centers) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= h * w) return;
    const float* z = logits + (int64_t)p * ld;
    const int32_t r = win / 2;
    int32_t best[2];
    for (int head = 0; head < 2; ++head) {
        const float* zh = z + head * nclass;
        const int32_t q = head == 0 ? qx : qy;
        float m = zh[0];
        for (int k = 1; k < q; ++k) m = fmaxf(m, zh[k]);
        float e[64], mass[64];
        for (int k = 0; k < q; ++k) e[k] = expf(zh[k] - m);
        float top = 0.f;
        for (int c = r; c <= q - 1 - r; ++c) {
            float s = 0.f;
            for (int k = c - r; k <= c + r; ++k) s += e[k];
            mass[c] = s;
            top = fmaxf(top, s);
        }
        int32_t b = r;
        for (int c = q - 1 - r; c >= r; --c)
            if (mass[c] >= top * (1.f - 1e-5f)) b = c;
        best[head] = b;
    }
    const int32_t cx = best[0], cy = best[1];
    const int32_t Y = p / w, X = p % w, W = 2 * w;
    for (int k = 0; k < 4; ++k) {
        const int64_t o = ((int64_t)(2 * Y + (k >> 1)) * W + 2 * X + (k & 1)) * 2;
        centers[o] = cx;
        centers[o + 1] = cy;
    }
}

// windows re-centred on a labelling: centre = label coordinates clamped so the box fits
__global__ void recenter_kernel(const int32_t* labels, int64_t n, int32_t qx, int32_t qy, int32_t win,
                                int32_t* centers) {
    const int32_t r = win / 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t lab = labels[i];
        centers[2 * i] = min(max(lab % qx, r), qx - 1 - r);
        centers[2 * i + 1] = min(max(lab / qx, r), qy - 1 - r);
    }
}

// class targets at half resolution: the label of the top-left pixel of each 2 x 2 block
__global__ void targets_kernel(const int32_t* labels, int32_t W, int32_t H, int32_t qx, int32_t* tx, int32_t* ty) {
    const int32_t w = W / 2, h = H / 2;
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= w * h) return;
    const int32_t lab = labels[(int64_t)(2 * (p / w)) * W + 2 * (p % w)];
    tx[p] = lab % qx;
    ty[p] = lab / qx;
}

int blocks_for(int64_t n, int per, int cap) {
    int64_t b = (n + per - 1) / per;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

template <int CIN, int COUT>
hipError_t run_conv(const uint16_t* in, const uint16_t* w, const float* bias, int32_t h, int32_t wd,
                    int32_t cout_real, int32_t relu, int32_t dil, const uint16_t* mask, int32_t ld, uint16_t* ob,
                    float* of, hipStream_t s) {
    const int64_t P = (int64_t)h * wd;
    hipLaunchKernelGGL((conv_kernel<CIN, COUT>), dim3((unsigned)((P + 63) / 64)), dim3(256), 0, s, in, w, bias, h,
                       wd, cout_real, relu, dil, mask, ld, ob, of);
    return hipGetLastError();
}

template <int CIN, int COUT>
hipError_t run_wgrad(const uint16_t* dy, const uint16_t* x, int32_t h, int32_t wd, int32_t cout_real, int32_t dil,
                     float* dw, hipStream_t s) {
    const int64_t nchunk = ((int64_t)h * wd + 31) / 32;
    int stripes = (int)((nchunk + 15) / 16);
    if (stripes > 64) stripes = 64;
    if (stripes < 1) stripes = 1;
    hipLaunchKernelGGL((wgrad_kernel<CIN, COUT>), dim3(9, stripes), dim3(256), 0, s, dy, x, h, wd, cout_real, dil, dw);
    return hipGetLastError();
}

}  // namespace cnn

using namespace cnn;

hipError_t launch_dsi_motion(const uint8_t* i0, const uint8_t* i1, int32_t W, int32_t H, int32_t r, int32_t cmax,
                             int32_t* out, hipStream_t s) {
    const int64_t n = (int64_t)W * H * (2 * r + 1) * (2 * r + 1);
    hipLaunchKernelGGL(dsi_motion_kernel, dim3(blocks_for(n, 256, 65536)), dim3(256), 0, s, i0, i1, W, H, r, cmax,
                       out);
    return hipGetLastError();
}

hipError_t launch_pool(const int32_t* cost, int32_t W, int32_t H, int32_t qx, int32_t qy, int32_t scale,
                       int32_t nbx, int32_t nch, int32_t mode, uint16_t* out, hipStream_t s) {
    const int64_t n = (int64_t)(W / 2) * (H / 2);
    if (qx * qy > POOL_QMAX) return hipErrorInvalidValue;
    const size_t lds = (size_t)4 * 4 * qx * qy * sizeof(int32_t);
    hipLaunchKernelGGL(pool_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), lds, s, cost, W, H, qx, qy, scale,
                       nbx, nch, mode, out);
    return hipGetLastError();
}

// (cin, cout) pairs compiled: the network's layers and their input gradients
hipError_t launch_conv(int32_t cin, int32_t cout_pad, const uint16_t* in, const uint16_t* w, const float* bias,
                       int32_t h, int32_t wd, int32_t cout_real, int32_t relu, int32_t dil, const uint16_t* mask,
                       int32_t ld, uint16_t* ob, float* of, hipStream_t s) {
    if (cin == 64 && cout_pad == 32) return run_conv<64, 32>(in, w, bias, h, wd, cout_real, relu, dil, mask, ld, ob, of, s);
    if (cin == 32 && cout_pad == 32) return run_conv<32, 32>(in, w, bias, h, wd, cout_real, relu, dil, mask, ld, ob, of, s);
    if (cin == 32 && cout_pad == 64) return run_conv<32, 64>(in, w, bias, h, wd, cout_real, relu, dil, mask, ld, ob, of, s);
    if (cin == 64 && cout_pad == 64) return run_conv<64, 64>(in, w, bias, h, wd, cout_real, relu, dil, mask, ld, ob, of, s);
    return hipErrorInvalidValue;
}

hipError_t launch_flip(const uint16_t* w, int32_t cin, int32_t cout, int32_t cout_pad, uint16_t* wt, hipStream_t s) {
    hipLaunchKernelGGL(flip_kernel, dim3(blocks_for((int64_t)cin * 9 * cout_pad, 256, 1024)), dim3(256), 0, s, w,
                       cin, cout, cout_pad, wt);
    return hipGetLastError();
}

hipError_t launch_wgrad(int32_t cin, int32_t cout_pad, const uint16_t* dy, const uint16_t* x, int32_t h, int32_t wd,
                        int32_t cout_real, int32_t dil, float* dw, hipStream_t s) {
    if (cin == 64 && cout_pad == 32) return run_wgrad<64, 32>(dy, x, h, wd, cout_real, dil, dw, s);
    if (cin == 32 && cout_pad == 32) return run_wgrad<32, 32>(dy, x, h, wd, cout_real, dil, dw, s);
    if (cin == 32 && cout_pad == 64) return run_wgrad<32, 64>(dy, x, h, wd, cout_real, dil, dw, s);
    if (cin == 64 && cout_pad == 64) return run_wgrad<64, 64>(dy, x, h, wd, cout_real, dil, dw, s);
    return hipErrorInvalidValue;
}

hipError_t launch_colsum(const float* a, int32_t rows, int32_t cols, int32_t ld, float* out, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3(blocks_for(rows, 4 * 64, 256)), dim3(256), 0, s, a, rows, cols, ld, out);
    return hipGetLastError();
}

hipError_t launch_ce(const float* logits, int32_t n, int32_t ld, const int32_t* tx, const int32_t* ty,
                     int32_t nclass, int32_t win, float* gf, uint16_t* gb, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(ce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, logits, n, ld, tx, ty, nclass,
                       win, gf, gb, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int32_t n, float lr, float b1,
                       float b2, float eps, float clip, int32_t t, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, s, p, g, m, v, pb, n, lr, b1, b2,
                       eps, c1, c2, clip);
    return hipGetLastError();
}

hipError_t launch_decode(const float* logits, int32_t h, int32_t w, int32_t ld, int32_t qx, int32_t qy, int32_t win,
                         int32_t nclass, int32_t* centers, hipStream_t s) {
    hipLaunchKernelGGL(decode_kernel, dim3(blocks_for((int64_t)h * w, 256, 1 << 20)), dim3(256), 0, s, logits, h, w,
                       ld, qx, qy, win, nclass, centers);
    return hipGetLastError();
}

hipError_t launch_recenter(const int32_t* labels, int64_t n, int32_t qx, int32_t qy, int32_t win, int32_t* centers,
                           hipStream_t s) {
    hipLaunchKernelGGL(recenter_kernel, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, labels, n, qx, qy, win,
                       centers);
    return hipGetLastError();
}

hipError_t launch_targets(const int32_t* labels, int32_t W, int32_t H, int32_t qx, int32_t* tx, int32_t* ty,
                          hipStream_t s) {
    hipLaunchKernelGGL(targets_kernel, dim3(blocks_for((int64_t)(W / 2) * (H / 2), 256, 1 << 20)), dim3(256), 0, s,
                       labels, W, H, qx, tx, ty);
    return hipGetLastError();
}

}  // namespace edp
