"""Pins of the label-window network reference: bf16 rounding against torch's conversion, the
convolution against scipy's correlation, gradients against finite differences, the cross
entropy's closed form at uniform logits, Adam's first step, pooling and decoding by hand."""
import numpy as np
import pytest
import torch
from scipy import signal

from oracle import cnn_ref as N


def test_bf16_matches_torch():
    x = np.random.default_rng(0).normal(0, 50, 4000).astype(np.float32)
    x[:4] = [0.0, -0.0, 1e-40, 3.0e38]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16(x), ref)


@pytest.mark.parametrize("dil", [1, 2, 3])
def test_conv_matches_scipy_correlate(dil):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(9, 11, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    out = N.conv3x3(x, w, b, dil)
    for co in range(4):
        k = np.zeros((2 * dil + 1, 2 * dil + 1, 3))
        k[::dil, ::dil] = w[co].transpose(0, 1, 2)          # dilated kernel: taps dil apart
        ref = b[co] + sum(signal.correlate2d(x[:, :, ci], k[:, :, ci], mode="same") for ci in range(3))
        assert np.allclose(out[:, :, co], ref)


def _fd(f, a, eps=1e-6):
    g = np.zeros_like(a)
    it = np.nditer(a, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = a[i]
        a[i] = old + eps
        fp = f()
        a[i] = old - eps
        fm = f()
        a[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


@pytest.mark.parametrize("dil", [1, 2])
def test_conv_backward_finite_differences(dil):
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 6, 3))
    w = rng.normal(size=(2, 3, 3, 3))
    dy = rng.normal(size=(5, 6, 2))
    f = lambda: float(np.sum(N.conv3x3(x, w, np.zeros(2), dil) * dy))
    dx, dw = N.conv3x3_backward(x, w, dy, dil)
    assert np.allclose(dx, _fd(f, x), atol=1e-5)
    assert np.allclose(dw, _fd(f, w), atol=1e-5)


@pytest.mark.parametrize("win", [1, 7])
def test_cross_entropy_closed_form_and_gradient(win):
    h, w = 3, 4
    tx = np.arange(12).reshape(h, w) % 31
    ty = (np.arange(12).reshape(h, w) * 7) % 31
    loss, g = N.ce_loss_grad(np.zeros((h, w, 62)), tx, ty, win=win)
    assert loss == pytest.approx(2 * np.log(31 / win))        # uniform: each window holds win / 31
    z = np.random.default_rng(3).normal(size=(h, w, 62))
    loss, g = N.ce_loss_grad(z, tx, ty, win=win)
    fd = _fd(lambda: N.ce_loss_grad(z, tx, ty, win=win)[0], z)
    assert np.allclose(g, fd, atol=1e-6)


def test_network_backward_finite_differences(monkeypatch):
    # with rounding switched off the gradient is exact and must match finite differences
    monkeypatch.setattr(N, "bf16", lambda a: np.asarray(a, dtype=np.float64))
    rng = np.random.default_rng(4)
    layers = ((4, 3), (3, 3), (3, 62))
    params = [{"w": rng.normal(0, 0.5, (co, 3, 3, ci)), "b": rng.normal(0, 0.1, co)} for ci, co in layers]
    x = rng.normal(size=(4, 4, 4))
    tx, ty = rng.integers(0, 31, (4, 4)), rng.integers(0, 31, (4, 4))

    def loss():
        z, _ = N.forward(x, params, (1, 2, 1))
        return N.ce_loss_grad(z, tx, ty)[0]

    z, acts = N.forward(x, params, (1, 2, 1))
    _, dz = N.ce_loss_grad(z, tx, ty)
    grads = N.backward(params, acts, dz, (1, 2, 1))
    for li in (0, 2):
        assert np.allclose(grads[li]["w"], _fd(loss, params[li]["w"]), atol=1e-6)
        assert np.allclose(grads[li]["b"], _fd(loss, params[li]["b"]), atol=1e-6)


def test_adam_first_step_is_a_signed_learning_rate():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    N.adam_step(p, g, m, v, 1, 0.01)
    assert np.allclose(p, [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01], atol=1e-6)


def test_adam_clip_limits_the_gradient():
    p = np.zeros(2)
    m, v = np.zeros(2), np.zeros(2)
    N.adam_step(p, np.array([5.0, -0.01]), m, v, 1, 0.1, clip=0.5)
    assert np.allclose(m, [0.05, -0.001])                 # (1 - b1) * clipped gradient
    assert np.allclose(p, [-0.1, 0.1], atol=1e-6)


def test_pool_by_hand():
    qx = qy = 5                       # blocks [0,4) and [4,5) per axis -> 4 channels
    cost = np.full((2, 2, 25), 100, np.int64)
    cost[0, 0, 0] = 20                # block (0,0) of pixel (0,0)
    cost[1, 1, 4 * 5 + 4] = 0         # block (1,1) of pixel (1,1)
    cost[0, 1, 2 * 5 + 4] = 60        # block (0,1) of pixel (0,1)
    out = N.pool_cost(cost, qx, qy, 100)
    assert out.shape == (1, 1, 4)
    assert out[0, 0, 0] == N.bf16((20 + 100 + 100 + 100) / 400.0)
    assert out[0, 0, 1] == N.bf16((100 + 60 + 100 + 100) / 400.0)
    assert out[0, 0, 2] == N.bf16(1.0)
    assert out[0, 0, 3] == N.bf16((100 + 100 + 100 + 0) / 400.0)


def test_axis_pool_by_hand():
    qx, qy = 3, 2
    cost = np.full((2, 2, 6), 50, np.int64)
    cost[0, 0, 1 * 3 + 2] = 10        # pixel (0,0): label column 2, row 1
    cost[1, 1, 0 * 3 + 0] = 30        # pixel (1,1): label column 0, row 0
    out = N.pool_cost(cost, qx, qy, 10, mode=1)
    assert out.shape == (1, 1, 64)
    assert out[0, 0, 0] == N.bf16((50 + 50 + 50 + 30) / 40.0)      # column 0
    assert out[0, 0, 2] == N.bf16((10 + 50 + 50 + 50) / 40.0)      # column 2
    assert out[0, 0, 3] == N.bf16((50 + 50 + 50 + 30) / 40.0)      # row 0
    assert out[0, 0, 4] == N.bf16((10 + 50 + 50 + 50) / 40.0)      # row 1
    assert out[0, 0, 1] == N.bf16(200 / 40.0) and np.all(out[0, 0, 5:] == 0)


def test_decode_by_hand():
    logits = np.zeros((1, 2, 62))
    logits[0, 0, 30] = 5.0            # column 30 -> the last window, centre 27
    logits[0, 0, 31 + 1] = 5.0        # row 1 -> the first window, centre 3
    logits[0, 1, 10] = 1.0
    logits[0, 1, 31 + 20] = 2.0
    c = N.decode(logits, 31, 31, 7)
    assert c.shape == (2, 4, 2)
    assert c[0, 0].tolist() == [27, 3] and c[1, 1].tolist() == [27, 3]
    assert c[0, 2].tolist() == [7, 17] and c[1, 3].tolist() == [7, 17]   # first window holding the peak
    # two peaks 6 apart: the window holding both wins over either alone
    z = np.full((1, 1, 62), -30.0)
    z[0, 0, 12] = z[0, 0, 18] = 3.0
    z[0, 0, 31 + 5] = 1.0
    assert N.decode(z, 31, 31, 7)[0, 0].tolist() == [15, 3]
