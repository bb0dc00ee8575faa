"""GPU parity of the data cost formation (edp_dsi: Sec. 2 eq. Cost_value, Sec. 5.1 eq. Cost_cmp)
against the oracle, bit-exact, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_1410_7922_amd as edp
import synth
from oracle import dsi_ref as D

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CASES = [
    # W, H, qx, qy, ox, oy, sx, sy, l2, cmax, composite, dtype
    (1, 1, 1, 1, 0, 0, 1, 1, 1, 10, False, torch.int16),
    (37, 5, 16, 1, 0, 0, -1, 1, 1, 50, False, torch.int16),
    (29, 11, 7, 1, 0, 0, -1, 1, 2, 10000, False, torch.int32),
    (40, 23, 5, 5, -2, -2, 1, 1, 2, 2500, False, torch.int32),
    (33, 17, 9, 3, -4, 1, 1, -1, 1, 90, False, torch.int16),
    (41, 9, 12, 1, 0, 0, -1, 1, 2, 10000, True, torch.int32),      # three-view stereo
    (26, 19, 7, 7, -3, -3, 1, 1, 2, 2500, True, torch.int32),      # three-view motion
    (17, 13, 3, 5, 2, -7, -1, 1, 1, 255, True, torch.int16),
    (64, 3, 100, 1, 10, 0, -1, 1, 1, 30000, False, torch.int16),   # labels reaching past the image
    # staged windows: 256-pixel segments, ragged last segment, segment starts off the 16-byte grid
    (300, 7, 9, 9, -4, -4, 1, 1, 2, 2500, True, torch.int32),
    (150, 4, 33, 1, 0, 0, -1, 1, 1, 50, False, torch.int16),
    (270, 3, 13, 1, 0, 0, -1, 1, 1, 40, False, torch.int16),
    (70, 2, 700, 1, -350, 0, 1, 1, 1, 255, True, torch.int16),     # 64-pixel segments, wide windows
    (200, 5, 31, 31, -15, -15, 1, 1, 2, 2500, False, torch.int32),  # the 961-label window shape
    # windows larger than 64 KB of LDS: the per-element kernel
    (40, 30, 1, 1100, 0, -550, 1, 1, 1, 90, False, torch.int16),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}q{c[2]}x{c[3]}l{c[8]}c{int(c[10])}")
def test_dsi_random_images(case):
    W, H, qx, qy, ox, oy, sx, sy, l2, cmax, comp, dt = case
    rng = np.random.default_rng(W * 7 + H)
    ims = [rng.integers(0, 256, (H, W), dtype=np.uint8) for _ in range(3)]
    ref = D.dsi(ims[0], ims[1], qx, qy, ox, oy, sx, sy, l2, cmax, i2=ims[2] if comp else None)
    note(f"dsi {W}x{H} q{qx}x{qy} l2 {l2} composite {comp} {dt}")
    got = edp.dsi(to_dev(ims[0]), to_dev(ims[1]), qx, qy, ox, oy, sx, sy, l2, cmax, dtype=dt,
                  i2=to_dev(ims[2]) if comp else None)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.int64), ref)


def test_dsi_unaligned_output():
    """An output that is not 16-byte aligned takes the element-by-element stores."""
    rng = np.random.default_rng(2)
    i0, i1 = (rng.integers(0, 256, (9, 21), dtype=np.uint8) for _ in range(2))
    ref = D.dsi(i0, i1, 6, 1, 0, 0, -1, 1, 1, 40)
    buf = torch.zeros(9 * 21 * 6 + 3, dtype=torch.int16, device=DEV)
    out = buf[3:].view(9, 21, 6)
    note("dsi unaligned output")
    edp.dsi(to_dev(i0), to_dev(i1), 6, 1, 0, 0, -1, 1, 1, 40, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), ref)
    assert (buf[:3].cpu().numpy() == 0).all()


def test_dsi_full_size_workloads():
    """The stereo 384x288 and motion 320x240 cost volumes of the workloads, from their frames."""
    p = synth.workload("stereo384x288")
    left, right = p.meta["frames"]
    note("dsi stereo384x288")
    got = edp.dsi(to_dev(left), to_dev(right), 32, 1, 0, 0, -1, 1, 1, 50, dtype=torch.int16)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), p.cost)
    m = synth.workload("motion320x240")
    i0, i1 = m.meta["frames"]
    note("dsi motion320x240")
    got = edp.dsi(to_dev(i0), to_dev(i1), 15, 15, -7, -7, 1, 1, 2, 2500, dtype=torch.int32)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), m.cost)


def test_dsi_961_label_volume_full_size():
    """The 961-label motion volume of the learned-window workload (640x480, int32, 1.18 GB) in the
    benchmark's call equals the workload generator's volume."""
    m = synth.workload("motion640x480")
    i0, i1 = m.meta["frames"]
    note("dsi motion640x480 961 labels")
    got = edp.dsi(to_dev(i0), to_dev(i1), 31, 31, -15, -15, 1, 1, 2, 2500, dtype=torch.int32)
    torch.cuda.synchronize()
    assert torch.equal(got, to_dev(m.cost))
