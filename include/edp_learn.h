/*
 * edp_learn.h -- C ABI of the label-window path of the MI355X EDP library:
 * a small convolutional network predicts, for every pixel, a window of labels
 * (its centre in the label space), and the EDP of Sec. 4.2 then runs over each
 * pixel's window only (edp_solve_windowed).  The plain EDP (edp_solve, edp.h)
 * stays the reference the windowed result is judged against.
 *
 * Conventions are those of edp.h: caller-owned device pointers, calls only
 * enqueue work on the given stream, argument errors are returned before
 * anything is enqueued, no allocation.  bf16 values are stored as uint16_t
 * (the upper half of an IEEE float32, round to nearest even).
 *
 * Network layout: activations channels-last [h][w][C] bf16; weights
 * [Cout][3][3][Cin] bf16 (float32 master copies held by the caller); biases
 * float32 [Cout]; logits and gradients float32 [h][w][ld].
 */
#ifndef EDP_LEARN_H
#define EDP_LEARN_H

#include <stddef.h>
#include <stdint.h>

#include "edp.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Motion cost volume (Sec. 2 eq. Cost_value with the squared difference and
 * truncation): C[y][x][q] = min((I0(x, y) - I1(x + dx, y + dy))^2, cmax) with
 * q = (dy + r)(2r + 1) + (dx + r), |dx|, |dy| <= r; a displaced position
 * outside the frame costs cmax.
 *   d_i0, d_i1  [H][W] uint8 frames;  d_cost [H][W][(2r+1)^2] int32 output
 */
edp_status edp_dsi_motion(const uint8_t* d_i0, const uint8_t* d_i1, int32_t W, int32_t H, int32_t r,
                          int32_t cmax, int32_t* d_cost, void* stream);

/*
 * Network input, bf16 [H/2][W/2][C]: per half-resolution pixel and channel a
 * minimum of the cost over a set of labels, summed over the 2 x 2 pixels and
 * divided in float32 by 4 * scale (scale >= 1).
 *   mode 0: C = ceil(qx/4) * ceil(qy/4) channels, one per block of 4 x 4 labels
 *   mode 1: C = 64 channels: the minimum over each label column (qx channels),
 *           then over each label row (qy channels), then zeros (qx + qy <= 64)
 *   d_cost [H][W][qy*qx] int32 (H, W even)
 */
edp_status edp_pool_cost(const int32_t* d_cost, int32_t W, int32_t H, int32_t qx, int32_t qy, int32_t scale,
                         int32_t mode, uint16_t* d_out, void* stream);

/*
 * 3x3 convolution with zero padding on the matrix cores (bf16 operands,
 * float32 accumulation): y[p][co] = b[co] + sum_{tap, ci} x[p + d tap][ci] w[co][tap][ci],
 * taps (dy, dx) in {-1, 0, 1}^2 scaled by the dilation d (1..64), optional ReLU.  cin in {32, 64}; cout <= 64, stored with ld = cout rounded up
 * to 32 or 64 (padded channels are written as 0).  d_b nullable.  Outputs:
 * d_y_bf16 and/or d_y_f32 (either nullable, not both).
 */
edp_status edp_conv3x3_forward(const uint16_t* d_x, const uint16_t* d_w, const float* d_b, int32_t h, int32_t w,
                               int32_t cin, int32_t cout, int32_t dilation, int32_t relu, uint16_t* d_y_bf16,
                               float* d_y_f32, void* stream);

/*
 * Input gradient of a 3x3 convolution layer whose input d_x was a ReLU output:
 * dx[p][ci] = [x[p][ci] > 0] * sum_{tap, co} dy[p - d tap][co] w[co][tap][ci].
 *   d_dy   [h][w][ld] bf16, ld = cout rounded up to 32 or 64
 *   d_wt   scratch of cin * 9 * ld bf16 (the flipped weights, written here)
 *   outputs [h][w][cin]: d_dx_f32 and d_dx_bf16 (both required)
 */
edp_status edp_conv3x3_dgrad(const uint16_t* d_dy, const uint16_t* d_w, const uint16_t* d_x, int32_t h,
                             int32_t w, int32_t cin, int32_t cout, int32_t dilation, uint16_t* d_wt,
                             float* d_dx_f32, uint16_t* d_dx_bf16, void* stream);

/*
 * Weight gradient, accumulated: dw[co][tap][ci] += sum_p dy[p][co] x[p + d tap][ci]
 * (d_dw float32 [cout][9][cin], cleared by the caller before the first call).
 */
edp_status edp_conv3x3_wgrad(const uint16_t* d_dy, const uint16_t* d_x, int32_t h, int32_t w, int32_t cin,
                             int32_t cout, int32_t dilation, float* d_dw, void* stream);

/* Bias gradient, accumulated: out[c] += sum_r a[r][c] for c < cols (cols <= 64). */
edp_status edp_colsum(const float* d_a, int32_t rows, int32_t cols, int32_t ld, float* d_out, void* stream);

/*
 * Window cross entropy of two heads of nclass logits per pixel (columns
 * [0, nclass) and [nclass, 2 nclass) of d_logits [n][ld]) against class targets
 * d_tx, d_ty [n]: per head -log of the softmax mass of the win labels around
 * the target (the window clamped into [0, nclass); win = 1 is the softmax cross
 * entropy).  *d_loss += mean over pixels of the sum over the heads; the
 * gradient, (p_k - [k in window] p_k / mass) / n, is written as float32 and
 * bf16 [n][ld] (columns past 2 nclass set to 0).
 */
edp_status edp_ce_loss(const float* d_logits, int32_t n, int32_t ld, const int32_t* d_tx, const int32_t* d_ty,
                       int32_t nclass, int32_t win, float* d_grad_f32, uint16_t* d_grad_bf16, float* d_loss,
                       void* stream);

/* One Adam step (bias-corrected, step t >= 1) over n float32 parameters, writing their bf16 copy.
 * Gradient elements are clipped to [-clip, clip] when clip > 0; non-finite ones count as 0. */
edp_status edp_adam(float* d_p, const float* d_g, float* d_m, float* d_v, uint16_t* d_p_bf16, int32_t n, float lr,
                    float beta1, float beta2, float eps, float clip, int32_t t, void* stream);

/*
 * Window centres from the logits [h][w][ld] of the half-resolution grid: for
 * each head (label column, label row) the centre c in [win/2, q-1-win/2] whose
 * window holds the largest softmax mass (the first such c), repeated over the
 * 2 x 2 full-resolution pixels: d_centers [2h][2w][2] = (cx, cy).
 */
edp_status edp_decode_windows(const float* d_logits, int32_t h, int32_t w, int32_t ld, int32_t qx, int32_t qy,
                              int32_t win, int32_t nclass, int32_t* d_centers, void* stream);

/* Windows re-centred on a labelling d_labels [H][W]: centre = the label's (column, row),
 * clamped to [win/2, q-1-win/2]; d_centers [H][W][2]. */
edp_status edp_window_recenter(const int32_t* d_labels, int32_t W, int32_t H, int32_t qx, int32_t qy, int32_t win,
                               int32_t* d_centers, void* stream);

/* Training targets: label columns / rows of the top-left pixel of each 2 x 2 block. */
edp_status edp_window_targets(const int32_t* d_labels, int32_t W, int32_t H, int32_t qx, int32_t* d_tx,
                              int32_t* d_ty, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* EDP_LEARN_H */
