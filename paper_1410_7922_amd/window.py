"""Label-window network: predicts, per pixel, the centre of a win x win label window.

Four 3x3 convolutions (64 -> 32 -> 32 -> 32 -> 2 x 31, ReLU between, dilations
1, 2, 4, 8) on the pooled cost volume at half resolution; bf16 weights and activations, float32
accumulation and master weights, trained with softmax cross entropy per label
axis and Adam.  Every operation runs in the library's kernels (edp_learn.h);
torch only allocates the buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B

LAYERS = ((64, 32), (32, 32), (32, 32), (32, 62))
DILATIONS = (1, 2, 4, 8)        # receptive field of 31 x 31 half-resolution pixels
NCLASS = 31


def _pad(c):
    return 32 if c <= 32 else 64


class WindowNet:
    """pool_mode: the network input (edp_pool_cost mode): 0 minima over 4 x 4 label blocks, 1 minima
    over label columns and rows."""

    def __init__(self, device, seed: int = 0, params: np.ndarray | None = None, pool_mode: int = 1):
        self.device = torch.device(device)
        self.pool_mode = pool_mode
        self.offsets = []            # (w offset, w size, b offset, b size) per layer in the flat vector
        n = 0
        for cin, cout in LAYERS:
            nw = cout * 9 * cin
            self.offsets.append((n, nw, n + nw, cout))
            n += nw + cout
        self.n = n
        if params is None:
            params = self.init_params(seed)
        self.p = torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(self.device)
        self.pb = torch.empty(n, dtype=torch.int16, device=self.device)
        self.g = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.t = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._refresh_bf16()
        self._bufs = {}

    # ---- parameters -----------------------------------------------------
    def init_params(self, seed):
        """He-uniform weights [Cout][3][3][Cin], zero biases, as one float32 vector."""
        rng = np.random.default_rng(seed)
        out = np.zeros(self.n, np.float32)
        for (cin, cout), (wo, nw, bo, nb) in zip(LAYERS, self.offsets):
            bound = np.sqrt(6.0 / (9 * cin))
            out[wo:wo + nw] = rng.uniform(-bound, bound, nw).astype(np.float32)
        return out

    def _refresh_bf16(self):
        # the bf16 copy comes from the Adam kernel itself: a step with zero gradient and zero
        # learning rate leaves the weights and moments unchanged and rounds the copy
        self.g.zero_()
        B.adam(self.p, self.g, self.m, self.v, self.pb, 0.0, 1)

    def layer(self, i):
        wo, nw, bo, nb = self.offsets[i]
        return self.pb[wo:wo + nw], self.p[bo:bo + nb], self.g[wo:wo + nw], self.g[bo:bo + nb]

    def params_numpy(self):
        return self.p.detach().cpu().numpy().copy()

    def save(self, path):
        np.savez(path, params=self.params_numpy(), layers=np.array(LAYERS, np.int32),
                 dilations=np.array(DILATIONS, np.int32), pool_mode=np.array(self.pool_mode, np.int32))

    @classmethod
    def load(cls, path, device):
        with np.load(path, allow_pickle=False) as f:
            mode = int(f["pool_mode"]) if "pool_mode" in f.files else 0
            return cls(device, params=f["params"], pool_mode=mode)

    # ---- buffers ----------------------------------------------------------
    def _buffers(self, h, w):
        key = (h, w)
        if key not in self._bufs:
            P = h * w
            d = self.device
            self._bufs[key] = {
                "acts": [torch.empty((h, w, _pad(cout)), dtype=torch.int16, device=d) for _, cout in LAYERS[:-1]],
                "logits": torch.empty((h, w, 64), dtype=torch.float32, device=d),
                "gf": [torch.empty((P, _pad(cout)), dtype=torch.float32, device=d) for _, cout in LAYERS],
                "gb": [torch.empty((P, _pad(cout)), dtype=torch.int16, device=d) for _, cout in LAYERS],
                "wt": torch.empty(64 * 9 * 64, dtype=torch.int16, device=d),
                "tx": torch.empty(P, dtype=torch.int32, device=d),
                "ty": torch.empty(P, dtype=torch.int32, device=d),
            }
        return self._bufs[key]

    # ---- network ----------------------------------------------------------
    def forward(self, x: torch.Tensor):
        """x [h][w][64] bf16 (int16 storage) -> logits [h][w][64] float32 (columns 62, 63 zero)."""
        h, w, _ = x.shape
        bufs = self._buffers(h, w)
        cur = x
        for i, (cin, cout) in enumerate(LAYERS):
            wb, b, _, _ = self.layer(i)
            if i + 1 < len(LAYERS):
                B.conv3x3_forward(cur, wb, b, h, w, cin, cout, True, y_bf16=bufs["acts"][i], dilation=DILATIONS[i])
                cur = bufs["acts"][i]
            else:
                B.conv3x3_forward(cur, wb, b, h, w, cin, cout, False, y_f32=bufs["logits"], dilation=DILATIONS[i])
        return bufs["logits"]

    def backward(self, x: torch.Tensor, tx: torch.Tensor, ty: torch.Tensor, win: int = 1):
        """Loss of the last forward() and the gradients (into self.g); returns the loss tensor.
        win > 1 trains the window mass around the target instead of the exact label."""
        h, w, _ = x.shape
        P = h * w
        bufs = self._buffers(h, w)
        self.g.zero_()
        self.loss.zero_()
        last = len(LAYERS) - 1
        B.ce_loss(bufs["logits"], P, 64, tx, ty, NCLASS, bufs["gf"][last], bufs["gb"][last], self.loss, win)
        inputs = [x] + bufs["acts"]
        for i in range(last, -1, -1):
            cin, cout = LAYERS[i]
            wb, _, gw, gbias = self.layer(i)
            B.colsum(bufs["gf"][i], P, cout, _pad(cout), gbias)
            B.conv3x3_wgrad(bufs["gb"][i], inputs[i], h, w, cin, cout, gw, dilation=DILATIONS[i])
            if i > 0:
                B.conv3x3_dgrad(bufs["gb"][i], wb, inputs[i], h, w, cin, cout, bufs["wt"],
                                bufs["gf"][i - 1], bufs["gb"][i - 1], dilation=DILATIONS[i])
        return self.loss

    def step(self, lr: float, clip: float = 1.0):
        self.t += 1
        B.adam(self.p, self.g, self.m, self.v, self.pb, lr, self.t, clip=clip)

    def train_step(self, x, tx, ty, lr, win: int = 1):
        self.forward(x)
        loss = self.backward(x, tx, ty, win)
        self.step(lr)
        return loss

    # ---- inference ----------------------------------------------------------
    def windows(self, cost: torch.Tensor, qx: int, qy: int, scale: int = 250, win: int = 7,
                pooled: torch.Tensor | None = None, centers: torch.Tensor | None = None):
        """Window centres [H][W][2] int32 for an int32 cost volume [H][W][qy*qx]; scale is the
        input normaliser the network was trained with."""
        H, W, _ = cost.shape
        x = B.pool_cost(cost, qx, qy, scale, out=pooled, mode=self.pool_mode)
        logits = self.forward(x)
        if centers is None:
            centers = torch.empty((H, W, 2), dtype=torch.int32, device=cost.device)
        B.decode_windows(logits, H // 2, W // 2, 64, qx, qy, win, NCLASS, centers)
        return centers

    def targets(self, labels: torch.Tensor, qx: int):
        H, W = labels.shape
        bufs = self._buffers(H // 2, W // 2)
        B.window_targets(labels, W, H, qx, bufs["tx"], bufs["ty"])
        return bufs["tx"], bufs["ty"]
