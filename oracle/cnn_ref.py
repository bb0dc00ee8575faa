"""Reference of the label-window network -- TEST INFRASTRUCTURE ONLY.

Float64 NumPy forward and backward of the small convolutional network that
predicts a per-pixel label window, on the same bf16-rounded operands the GPU
kernels use (bf16 weights and activations, float accumulation).  Only tests
and the smoke check import this module; it shares no code with the library.

Network (per pixel of the half-resolution grid, channels last):
  input   pooled cost volume: for each label block of 4 x 4 labels the minimum
          cost over the block, summed over the 2 x 2 pixels, divided (float32)
          by 4 x a scale, rounded to bf16 (64 channels for 31 x 31 labels)
  conv3x3 64 -> 32, ReLU;  conv3x3 32 -> 32, ReLU;  conv3x3 32 -> 32, ReLU;
  conv3x3 32 -> 2 * 31 logits (first half: label column, second: label row)
  dilations 1, 2, 4, 8; zero padding; weights [Cout][3][3][Cin] (bf16), bias
  [Cout] (float32)
Training: per head the negative log softmax mass of the window of labels
around the label of the top-left pixel of each 2 x 2 block (a window of one
label is the softmax cross entropy), averaged over pixels and summed over the
heads; Adam on float32 master weights.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def label_blocks(q: int, block: int = 4):
    """Label index ranges [lo, hi) of the pooling blocks along one label axis."""
    return [(s, min(s + block, q)) for s in range(0, q, block)]


def pool_cost(cost, qx, qy, scale, block=4, mode=0):
    """cost [H][W][qy*qx] (H, W even) -> float64 [H/2][W/2][C], bf16-rounded.  mode 0: one channel per
    block x block labels; mode 1: 64 channels, the minimum over each label column, then over each
    label row, then zeros."""
    H, W, Q = cost.shape
    assert Q == qx * qy and H % 2 == 0 and W % 2 == 0
    c = np.asarray(cost, dtype=np.int64).reshape(H, W, qy, qx)
    if mode == 0:
        bx, by = label_blocks(qx, block), label_blocks(qy, block)
        sets = [(y0, y1, x0, x1) for (y0, y1) in by for (x0, x1) in bx]
        nch = len(sets)
    else:
        sets = [(0, qy, x, x + 1) for x in range(qx)] + [(y, y + 1, 0, qx) for y in range(qy)]
        nch = 64
    out = np.zeros((H // 2, W // 2, nch), np.float64)
    for ch, (y0, y1, x0, x1) in enumerate(sets):
        m = c[:, :, y0:y1, x0:x1].min(axis=(2, 3))               # [H][W]
        s = m[0::2, 0::2] + m[0::2, 1::2] + m[1::2, 0::2] + m[1::2, 1::2]
        # one correctly rounded float32 division of two exact integers
        out[:, :, ch] = s.astype(np.float32) / np.float32(4 * scale)
    return bf16(out)


def conv3x3(x, w, b, dil=1):
    """x [h][w][cin], w [cout][3][3][cin], b [cout] -> [h][w][cout] (zero padding, taps dil apart)."""
    h, wd, cin = x.shape
    cout = w.shape[0]
    xp = np.zeros((h + 2 * dil, wd + 2 * dil, cin))
    xp[dil:dil + h, dil:dil + wd] = x
    out = np.zeros((h, wd, cout)) + b
    for dy in range(3):
        for dx in range(3):
            out += xp[dy * dil:dy * dil + h, dx * dil:dx * dil + wd] @ w[:, dy, dx, :].T
    return out


def conv3x3_backward(x, w, dy_, dil=1):
    """Gradients of conv3x3 w.r.t. its input and weights for output gradient dy_."""
    h, wd, cin = x.shape
    xp = np.zeros((h + 2 * dil, wd + 2 * dil, cin))
    xp[dil:dil + h, dil:dil + wd] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            sl = (slice(dy * dil, dy * dil + h), slice(dx * dil, dx * dil + wd))
            dxp[sl] += dy_ @ w[:, dy, dx, :]
            dw[:, dy, dx, :] = np.einsum("hwo,hwi->oi", dy_, xp[sl])
    return dxp[dil:dil + h, dil:dil + wd], dw


LAYERS = ((64, 32), (32, 32), (32, 32), (32, 62))
DILATIONS = (1, 2, 4, 8)


def init_params(rng, layers=LAYERS):
    """He-uniform float32 master weights [Cout][3][3][Cin] and zero biases."""
    params = []
    for cin, cout in layers:
        bound = np.sqrt(6.0 / (9 * cin))
        params.append({"w": rng.uniform(-bound, bound, (cout, 3, 3, cin)).astype(np.float32),
                       "b": np.zeros(cout, np.float32)})
    return params


def forward(x, params, dilations=DILATIONS):
    """Returns (logits [h][w][62] float64, inputs of every layer (bf16-rounded))."""
    acts = [bf16(x)]
    for li, p in enumerate(params):
        z = conv3x3(acts[-1], bf16(p["w"]), np.asarray(p["b"], np.float64), dilations[li])
        if li + 1 < len(params):
            acts.append(bf16(np.maximum(z, 0.0)))
        else:
            return z, acts
    raise AssertionError


def targets(labels, qx):
    """Class targets of the half-resolution grid: the top-left label of each 2 x 2 block."""
    lab = np.asarray(labels)[0::2, 0::2]
    return lab % qx, lab // qx


def ce_loss_grad(logits, tx, ty, nclass=31, win=1):
    """Mean over pixels of the two heads' window cross entropies -log(softmax mass of the win labels
    around the target, the window clamped into the label range), and its logit gradient.  win = 1
    is the softmax cross entropy."""
    h, w, _ = logits.shape
    n = h * w
    r = win // 2
    loss = 0.0
    grad = np.zeros_like(logits)
    for head, t in ((0, tx), (1, ty)):
        z = logits[:, :, head * nclass:(head + 1) * nclass]
        e = np.exp(z - z.max(axis=2, keepdims=True))
        p = e / e.sum(axis=2, keepdims=True)
        c = np.clip(np.asarray(t), r, nclass - 1 - r)
        k = np.arange(nclass)[None, None, :]
        inwin = np.abs(k - c[:, :, None]) <= r
        mass = np.sum(p * inwin, axis=2)
        loss += float(np.sum(-np.log(mass))) / n
        grad[:, :, head * nclass:(head + 1) * nclass] = (p - p * inwin / mass[:, :, None]) / n
    return loss, grad


def backward(params, acts, dlogits, dilations=DILATIONS):
    """Gradients of every layer.  The output gradient of a layer enters the products rounded to
    bf16 (as the GPU's matrix operands); bias gradients use it unrounded."""
    grads = [None] * len(params)
    d = dlogits
    for li in range(len(params) - 1, -1, -1):
        p = params[li]
        db = d.sum(axis=(0, 1))
        dx, dw = conv3x3_backward(acts[li], bf16(p["w"]), bf16(d), dilations[li])
        grads[li] = {"w": dw, "b": db}
        if li > 0:
            d = dx * (acts[li] > 0)
    return grads


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, clip=0.0):
    """One Adam update (bias-corrected) of the float master weights, in place; gradient elements
    clipped to [-clip, clip] when clip > 0."""
    if clip > 0:
        g = np.clip(g, -clip, clip)
    m[:] = b1 * m + (1 - b1) * g
    v[:] = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p[:] = p - lr * mh / (np.sqrt(vh) + eps)


def window_mass(logits_head, q, win):
    """Mass sum_{|k-c| <= win/2} exp(z_k - max z) of every admissible window [h][w][q - win + 1]."""
    z = logits_head[:, :, :q]
    e = np.exp(z - z.max(axis=2, keepdims=True))
    return np.stack([e[:, :, c:c + win].sum(axis=2) for c in range(q - win + 1)], axis=2)


def decode(logits, qx, qy, win, nclass=31, rel=1e-5):
    """Window centres at full resolution [2h][2w][2] = (cx, cy): per head the first centre whose
    window mass is within a factor (1 - rel) of the largest, repeated over each 2 x 2 block."""
    r = win // 2
    out = []
    for head, q in ((0, qx), (1, qy)):
        m = window_mass(logits[:, :, head * nclass:(head + 1) * nclass], q, win)
        ok = m >= m.max(axis=2, keepdims=True) * (1 - rel)
        out.append(np.argmax(ok, axis=2) + r)
    c = np.stack(out, axis=-1)
    return np.repeat(np.repeat(c, 2, axis=0), 2, axis=1).astype(np.int32)


def recenter(labels, qx, qy, win):
    """Window centres [H][W][2] = (cx, cy) re-centred on a labelling: each label's column and row,
    clamped so the win x win window stays inside the qx x qy label space."""
    lab = np.asarray(labels, dtype=np.int64)
    r = win // 2
    cx = np.clip(lab % qx, r, qx - 1 - r)
    cy = np.clip(lab // qx, r, qy - 1 - r)
    return np.stack([cx, cy], axis=-1).astype(np.int32)


def params_from_flat(flat, layers=LAYERS):
    """Per-layer weights [Cout][3][3][Cin] and biases [Cout] from one flat float32 vector that holds,
    layer after layer, the weights then the biases."""
    flat = np.asarray(flat, dtype=np.float32)
    out, n = [], 0
    for cin, cout in layers:
        nw = cout * 9 * cin
        out.append({"w": flat[n:n + nw].reshape(cout, 3, 3, cin), "b": flat[n + nw:n + nw + cout]})
        n += nw + cout
    assert n == flat.size, "parameter vector does not match the layers"
    return out


def network_centres(cost, qx, qy, params, scale, win, pool_mode=1):
    """Window centres [H][W][2] the network proposes for an int32 cost volume [H][W][qy*qx]: the
    pooled input, the forward pass and the window decoding above."""
    x = pool_cost(cost, qx, qy, scale, mode=pool_mode)
    logits, _ = forward(x, params)
    return decode(logits, qx, qy, win)
