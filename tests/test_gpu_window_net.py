"""GPU checks of the label-window network kernels against the float64 reference (oracle/cnn_ref):
the matrix-core convolution, its input and weight gradients, bias gradient, cross entropy, Adam,
decoding, targets (within float32-accumulation tolerances where rounding order differs, exact
where the computation is integer or a selection), the pooled input and the motion cost volume
(bit-exact), and a few training steps that lower the loss."""
import numpy as np
import pytest
import torch

import paper_1410_7922_amd as edp
from paper_1410_7922_amd import binding as B
from paper_1410_7922_amd.window import LAYERS, WindowNet
import synth
from oracle import cnn_ref as N

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def to_bf16_dev(a):
    """float array (already bf16-representable) -> device int16 storage of its bf16 bits"""
    t = torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).contiguous().to(DEV)


def from_bf16_dev(t):
    return t.cpu().view(torch.bfloat16).to(torch.float64).numpy()


def pad(c):
    return 32 if c <= 32 else 64


@pytest.mark.parametrize("cin,cout,dil", [(64, 32, 1), (32, 32, 2), (32, 62, 8), (64, 64, 4), (32, 32, 16)])
def test_conv_forward_matches_reference(cin, cout, dil):
    note(f"conv forward {cin}->{cout} dilation {dil}")
    rng = np.random.default_rng(cin * 100 + cout)
    h, w = 9, 13                                    # 117 pixels: two workgroups, ragged
    x = N.bf16(rng.normal(0, 1, (h, w, cin)))
    wt = N.bf16(rng.normal(0, 0.2, (cout, 3, 3, cin)))
    b = rng.normal(0, 0.1, cout).astype(np.float32)
    ref = N.conv3x3(x, wt, b.astype(np.float64), dil)
    yf = torch.empty((h, w, pad(cout)), dtype=torch.float32, device=DEV)
    B.conv3x3_forward(to_bf16_dev(x), to_bf16_dev(wt), torch.from_numpy(b).to(DEV), h, w, cin, cout, False, y_f32=yf,
                      dilation=dil)
    yb = torch.empty((h, w, pad(cout)), dtype=torch.int16, device=DEV)
    B.conv3x3_forward(to_bf16_dev(x), to_bf16_dev(wt), torch.from_numpy(b).to(DEV), h, w, cin, cout, True, y_bf16=yb,
                      dilation=dil)
    torch.cuda.synchronize()
    got = yf.cpu().numpy()
    assert np.allclose(got[:, :, :cout], ref, rtol=1e-4, atol=1e-4)
    assert np.all(got[:, :, cout:] == 0)
    gb = from_bf16_dev(yb)[:, :, :cout]
    rb = N.bf16(np.maximum(ref, 0))
    # identical up to a rounding-boundary difference of one bf16 step
    assert np.allclose(gb, rb, rtol=2 ** -7, atol=1e-6)


@pytest.mark.parametrize("cin,cout,dil", [(32, 32, 1), (32, 62, 8), (64, 32, 2), (32, 32, 4)])
def test_conv_gradients_match_reference(cin, cout, dil):
    note(f"conv gradients {cin}->{cout} dilation {dil}")
    rng = np.random.default_rng(7 + cin + cout)
    h, w = 11, 7
    P = h * w
    x = N.bf16(np.maximum(rng.normal(0, 1, (h, w, cin)), 0))       # a ReLU output: mask matters
    wt = N.bf16(rng.normal(0, 0.2, (cout, 3, 3, cin)))
    d = rng.normal(0, 1e-2, (h, w, cout))
    dx_ref, dw_ref = N.conv3x3_backward(x, wt, N.bf16(d), dil)
    dx_ref = dx_ref * (x > 0)
    dpad = np.zeros((h, w, pad(cout)))
    dpad[:, :, :cout] = d
    dyb = to_bf16_dev(N.bf16(dpad))
    scratch = torch.empty(64 * 9 * 64, dtype=torch.int16, device=DEV)
    dxf = torch.empty((P, cin), dtype=torch.float32, device=DEV)
    dxb = torch.empty((P, cin), dtype=torch.int16, device=DEV)
    B.conv3x3_dgrad(dyb, to_bf16_dev(wt), to_bf16_dev(x), h, w, cin, cout, scratch, dxf, dxb, dilation=dil)
    dw = torch.zeros((cout, 9, cin), dtype=torch.float32, device=DEV)
    B.conv3x3_wgrad(dyb, to_bf16_dev(x), h, w, cin, cout, dw, dilation=dil)
    db = torch.zeros(cout, dtype=torch.float32, device=DEV)
    df = torch.from_numpy(dpad.reshape(P, -1).astype(np.float32)).to(DEV)
    B.colsum(df, P, cout, pad(cout), db)
    torch.cuda.synchronize()
    assert np.allclose(dxf.cpu().numpy().reshape(h, w, cin), dx_ref, rtol=1e-4, atol=1e-6)
    assert np.allclose(from_bf16_dev(dxb).reshape(h, w, cin), N.bf16(dx_ref), rtol=2 ** -7, atol=1e-8)
    assert np.allclose(dw.cpu().numpy().reshape(cout, 3, 3, cin), dw_ref, rtol=1e-4, atol=1e-5)
    assert np.allclose(db.cpu().numpy(), d.sum(axis=(0, 1)), rtol=1e-4, atol=1e-5)


def test_cross_entropy_adam_decode_targets():
    note("cross entropy, adam, decode, targets")
    rng = np.random.default_rng(5)
    h, w = 6, 10
    P = h * w
    z = np.zeros((h, w, 64), np.float32)
    z[:, :, :62] = rng.normal(0, 2, (h, w, 62))
    tx, ty = rng.integers(0, 31, (h, w)), rng.integers(0, 31, (h, w))
    zt = torch.from_numpy(z).to(DEV)
    txd = torch.from_numpy(tx.astype(np.int32).ravel()).to(DEV)
    tyd = torch.from_numpy(ty.astype(np.int32).ravel()).to(DEV)
    for win in (1, 7):
        loss_ref, g_ref = N.ce_loss_grad(z[:, :, :62].astype(np.float64), tx, ty, win=win)
        gf = torch.empty((P, 64), dtype=torch.float32, device=DEV)
        gb = torch.empty((P, 64), dtype=torch.int16, device=DEV)
        loss = torch.zeros(1, dtype=torch.float32, device=DEV)
        B.ce_loss(zt, P, 64, txd, tyd, 31, gf, gb, loss, win)
        torch.cuda.synchronize()
        assert float(loss.item()) == pytest.approx(loss_ref, rel=1e-5)
        assert np.allclose(gf.cpu().numpy().reshape(h, w, 64)[:, :, :62], g_ref, rtol=1e-4, atol=1e-7)
        assert np.all(gf.cpu().numpy().reshape(h, w, 64)[:, :, 62:] == 0)
    # Adam: three steps against the reference
    p = rng.normal(0, 1, 1000).astype(np.float32)
    pd, m, v = torch.from_numpy(p.copy()).to(DEV), torch.zeros(1000, device=DEV), torch.zeros(1000, device=DEV)
    pbd = torch.empty(1000, dtype=torch.int16, device=DEV)
    pr, mr, vr = p.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for t in (1, 2, 3):
        g = rng.normal(0, 1e-2, 1000).astype(np.float32)
        B.adam(pd, torch.from_numpy(g).to(DEV), m, v, pbd, 1e-3, t, clip=0.015)
        N.adam_step(pr, g.astype(np.float64), mr, vr, t, 1e-3, clip=0.015)
    torch.cuda.synchronize()
    assert np.allclose(pd.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    assert np.array_equal(from_bf16_dev(pbd), N.bf16(pd.cpu().numpy()))
    # decode: same logits -> same centres
    cen = torch.empty((2 * h, 2 * w, 2), dtype=torch.int32, device=DEV)
    B.decode_windows(zt, h, w, 64, 31, 31, 7, 31, cen)
    torch.cuda.synchronize()
    assert np.array_equal(cen.cpu().numpy(), N.decode(z.astype(np.float64), 31, 31, 7))
    # targets
    lab = rng.integers(0, 961, (2 * h, 2 * w)).astype(np.int32)
    B.window_targets(torch.from_numpy(lab).to(DEV), 2 * w, 2 * h, 31, txd, tyd)
    torch.cuda.synchronize()
    rx, ry = N.targets(lab, 31)
    assert np.array_equal(txd.cpu().numpy().reshape(h, w), rx) and np.array_equal(tyd.cpu().numpy().reshape(h, w), ry)


def test_motion_cost_and_pool_bit_exact():
    note("motion cost volume and pooled input")
    i0, i1, _, _ = synth.motion_frames(seed=11, W=48, H=36, r=15)
    ref = synth.motion_cost(i0, i1, 15, 2500)
    cost = B.dsi_motion(torch.from_numpy(i0).to(DEV), torch.from_numpy(i1).to(DEV), 15, 2500)
    torch.cuda.synchronize()
    assert np.array_equal(cost.cpu().numpy(), ref)
    for mode in (0, 1):
        pooled = B.pool_cost(cost, 31, 31, 250, mode=mode)
        torch.cuda.synchronize()
        assert np.array_equal(from_bf16_dev(pooled), N.pool_cost(ref, 31, 31, 250, mode=mode))


def _ref_params(net):
    flat = net.params_numpy()
    out = []
    for (cin, cout), (wo, nw, bo, nb) in zip(LAYERS, net.offsets):
        out.append({"w": flat[wo:wo + nw].reshape(cout, 3, 3, cin), "b": flat[bo:bo + nb]})
    return out


def _term_magnitudes(params, acts, dz, dilations=(1, 2, 4, 8)):
    """Per gradient element, an upper bound of the sum of the magnitudes of the products it adds up:
    the reference's backward pass with every operand replaced by its magnitude (the upstream
    gradient's magnitudes propagated through |W| and the ReLU masks)."""
    out = [None] * len(params)
    a = np.abs(dz)
    for li in range(len(params) - 1, -1, -1):
        wb = np.abs(N.bf16(params[li]["w"]))
        dx_abs, dw_abs = N.conv3x3_backward(np.abs(acts[li]), wb, a, dilations[li])
        out[li] = {"w": dw_abs, "b": a.sum(axis=(0, 1))}
        if li > 0:
            a = dx_abs * (acts[li] > 0)
    return out


def test_network_step_matches_reference():
    """One forward and backward pass of the whole network, element by element.  Every layer of the
    reference runs on the GPU's own bf16 input for that layer (its stored activations), so both
    sides take the same ReLU decisions.  An activation may then differ by one bf16 step (where the
    float32 and float64 sums round to different neighbours), the logits by float32 rounding, and a
    gradient element by a few bf16 units of the sum of its terms' magnitudes: the gradient reaching
    layer l has been rounded to bf16 at most 4 - l times on the way down, each rounding moving an
    element by at most 2^-8 of its magnitude bound, so 2^-6 of that sum bounds every layer."""
    note("network forward / backward / step")
    rng = np.random.default_rng(9)
    h, w = 10, 14
    x = N.bf16(rng.uniform(0, 1, (h, w, 64)))
    tx, ty = rng.integers(0, 31, (h, w)), rng.integers(0, 31, (h, w))
    net = WindowNet(DEV, seed=3)
    params = _ref_params(net)
    xd = to_bf16_dev(x)
    z = net.forward(xd)
    loss = net.backward(xd, torch.from_numpy(tx.astype(np.int32).ravel()).to(DEV),
                        torch.from_numpy(ty.astype(np.int32).ravel()).to(DEV))
    torch.cuda.synchronize()
    bufs = net._buffers(h, w)
    acts = [x] + [from_bf16_dev(a)[:, :, :cout] for a, (_, cout) in zip(bufs["acts"], LAYERS[:-1])]
    dil = (1, 2, 4, 8)
    zg = z.cpu().numpy()[:, :, :62].astype(np.float64)
    for li, p in enumerate(params):
        zr = N.conv3x3(acts[li], N.bf16(p["w"]), np.asarray(p["b"], np.float64), dil[li])
        if li + 1 < len(params):
            assert np.allclose(acts[li + 1], N.bf16(np.maximum(zr, 0.0)), rtol=2 ** -7, atol=1e-6), li
        else:
            assert np.allclose(zg, zr, rtol=1e-4, atol=1e-4)
    loss_ref, dz = N.ce_loss_grad(zg, tx, ty)
    assert float(loss.item()) == pytest.approx(loss_ref, rel=1e-5)
    grads = N.backward(params, acts, dz)
    mags = _term_magnitudes(params, acts, dz)
    g = net.g.cpu().numpy()
    for li, (wo, nw, bo, nb) in enumerate(net.offsets):
        for key, off, n in (("w", wo, nw), ("b", bo, nb)):
            ref = grads[li][key].ravel()
            bound = 2.0 ** -6 * mags[li][key].ravel() + 1e-9
            err = np.abs(g[off:off + n] - ref)
            worst = int(np.argmax(err / bound))
            assert np.all(err <= bound), (li, key, worst, g[off + worst], ref[worst], bound[worst])


def test_training_lowers_the_loss():
    note("training steps")
    p = synth.motion_problem(seed=21, W=64, H=48, r=15)
    cost = torch.from_numpy(p.cost).to(DEV)
    labels = torch.from_numpy(p.meta["gt"].astype(np.int32)).to(DEV)
    net = WindowNet(DEV, seed=1)
    x = B.pool_cost(cost, 31, 31, 2500)
    tx, ty = net.targets(labels, 31)
    losses = [float(net.train_step(x, tx, ty, 3e-3).item()) for _ in range(60)]
    torch.cuda.synchronize()
    assert losses[-1] < 0.7 * losses[0], losses[::10]
