// C ABI of the label-window network kernels (argument checks, launches).
#include <hip/hip_runtime.h>

#include "../../include/edp_learn.h"
#include "edp_internal.hpp"

using namespace edp;

namespace {

edp_status st(hipError_t e) { return e == hipSuccess ? EDP_OK : EDP_E_HIP; }
int32_t pad_channels(int32_t c) { return c <= 32 ? 32 : 64; }
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" {

edp_status edp_dsi_motion(const uint8_t* d_i0, const uint8_t* d_i1, int32_t W, int32_t H, int32_t r, int32_t cmax,
                          int32_t* d_cost, void* stream) {
    if (!d_i0 || !d_i1 || !d_cost || W < 1 || H < 1 || r < 0 || r > 31 || cmax < 0) return EDP_E_INVALID;
    return st(launch_dsi_motion(d_i0, d_i1, W, H, r, cmax, d_cost, (hipStream_t)stream));
}

edp_status edp_pool_cost(const int32_t* d_cost, int32_t W, int32_t H, int32_t qx, int32_t qy, int32_t scale,
                         int32_t mode, uint16_t* d_out, void* stream) {
    if (!d_cost || !d_out || W < 2 || H < 2 || (W & 1) || (H & 1) || qx < 1 || qy < 1 || scale < 1 ||
        (mode != 0 && mode != 1))
        return EDP_E_INVALID;
    const int32_t nbx = (qx + 3) / 4, nby = (qy + 3) / 4;
    if (mode == 0 && nbx * nby > 64) return EDP_E_UNSUPPORTED;
    if (mode == 1 && qx + qy > 64) return EDP_E_UNSUPPORTED;
    return st(launch_pool(d_cost, W, H, qx, qy, scale, nbx, mode == 0 ? nbx * nby : 64, mode, d_out,
                          (hipStream_t)stream));
}

edp_status edp_conv3x3_forward(const uint16_t* d_x, const uint16_t* d_w, const float* d_b, int32_t h, int32_t w,
                               int32_t cin, int32_t cout, int32_t dilation, int32_t relu, uint16_t* d_y_bf16,
                               float* d_y_f32, void* stream) {
    if (!d_x || !d_w || h < 1 || w < 1 || (cin != 32 && cin != 64) || cout < 1 || cout > 64 || dilation < 1 ||
        dilation > 64)
        return EDP_E_INVALID;
    if ((!d_y_bf16) == (!d_y_f32)) return EDP_E_INVALID;
    if (!aligned16(d_x) || !aligned16(d_w)) return EDP_E_INVALID;
    const int32_t ld = pad_channels(cout);
    return st(launch_conv(cin, ld, d_x, d_w, d_b, h, w, cout, relu ? 1 : 0, dilation, nullptr, ld, d_y_bf16, d_y_f32,
                          (hipStream_t)stream));
}

edp_status edp_conv3x3_dgrad(const uint16_t* d_dy, const uint16_t* d_w, const uint16_t* d_x, int32_t h, int32_t w,
                             int32_t cin, int32_t cout, int32_t dilation, uint16_t* d_wt, float* d_dx_f32,
                             uint16_t* d_dx_bf16, void* stream) {
    if (!d_dy || !d_w || !d_x || !d_wt || !d_dx_f32 || !d_dx_bf16 || h < 1 || w < 1 || (cin != 32 && cin != 64) ||
        cout < 1 || cout > 64 || dilation < 1 || dilation > 64)
        return EDP_E_INVALID;
    if (!aligned16(d_dy) || !aligned16(d_wt)) return EDP_E_INVALID;
    const int32_t ld = pad_channels(cout);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_flip(d_w, cin, cout, ld, d_wt, s);
    if (e == hipSuccess)
        e = launch_conv(ld, cin, d_dy, d_wt, nullptr, h, w, cin, 0, dilation, d_x, cin, d_dx_bf16, d_dx_f32, s);
    return st(e);
}

edp_status edp_conv3x3_wgrad(const uint16_t* d_dy, const uint16_t* d_x, int32_t h, int32_t w, int32_t cin,
                             int32_t cout, int32_t dilation, float* d_dw, void* stream) {
    if (!d_dy || !d_x || !d_dw || h < 1 || w < 1 || (cin != 32 && cin != 64) || cout < 1 || cout > 64 ||
        dilation < 1 || dilation > 64)
        return EDP_E_INVALID;
    return st(launch_wgrad(cin, pad_channels(cout), d_dy, d_x, h, w, cout, dilation, d_dw, (hipStream_t)stream));
}

edp_status edp_colsum(const float* d_a, int32_t rows, int32_t cols, int32_t ld, float* d_out, void* stream) {
    if (!d_a || !d_out || rows < 1 || cols < 1 || cols > 64 || ld < cols) return EDP_E_INVALID;
    return st(launch_colsum(d_a, rows, cols, ld, d_out, (hipStream_t)stream));
}

edp_status edp_ce_loss(const float* d_logits, int32_t n, int32_t ld, const int32_t* d_tx, const int32_t* d_ty,
                       int32_t nclass, int32_t win, float* d_grad_f32, uint16_t* d_grad_bf16, float* d_loss,
                       void* stream) {
    if (!d_logits || !d_tx || !d_ty || !d_grad_f32 || !d_grad_bf16 || n < 1 || nclass < 1 || 2 * nclass > ld ||
        win < 1 || !(win & 1) || win > nclass)
        return EDP_E_INVALID;
    return st(launch_ce(d_logits, n, ld, d_tx, d_ty, nclass, win, d_grad_f32, d_grad_bf16, d_loss,
                        (hipStream_t)stream));
}

edp_status edp_adam(float* d_p, const float* d_g, float* d_m, float* d_v, uint16_t* d_p_bf16, int32_t n, float lr,
                    float beta1, float beta2, float eps, float clip, int32_t t, void* stream) {
    if (!d_p || !d_g || !d_m || !d_v || !d_p_bf16 || n < 1 || t < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !(clip >= 0.f))
        return EDP_E_INVALID;
    return st(launch_adam(d_p, d_g, d_m, d_v, d_p_bf16, n, lr, beta1, beta2, eps, clip, t, (hipStream_t)stream));
}

edp_status edp_decode_windows(const float* d_logits, int32_t h, int32_t w, int32_t ld, int32_t qx, int32_t qy,
                              int32_t win, int32_t nclass, int32_t* d_centers, void* stream) {
    if (!d_logits || !d_centers || h < 1 || w < 1 || nclass < 1 || 2 * nclass > ld || win < 1 || !(win & 1) ||
        win > qx || win > qy || qx > nclass || qy > nclass)
        return EDP_E_INVALID;
    return st(launch_decode(d_logits, h, w, ld, qx, qy, win, nclass, d_centers, (hipStream_t)stream));
}

edp_status edp_window_targets(const int32_t* d_labels, int32_t W, int32_t H, int32_t qx, int32_t* d_tx,
                              int32_t* d_ty, void* stream) {
    if (!d_labels || !d_tx || !d_ty || W < 2 || H < 2 || qx < 1) return EDP_E_INVALID;
    return st(launch_targets(d_labels, W, H, qx, d_tx, d_ty, (hipStream_t)stream));
}

edp_status edp_window_recenter(const int32_t* d_labels, int32_t W, int32_t H, int32_t qx, int32_t qy, int32_t win,
                               int32_t* d_centers, void* stream) {
    if (!d_labels || !d_centers || W < 1 || H < 1 || win < 1 || !(win & 1) || win > qx || win > qy)
        return EDP_E_INVALID;
    return st(launch_recenter(d_labels, (int64_t)W * H, qx, qy, win, d_centers, (hipStream_t)stream));
}

}  // extern "C"
