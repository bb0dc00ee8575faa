"""edp_solve_static (edp_solve with its workspace in the library's static device array, for callers
that cannot allocate) through the C ABI against edp_solve on the same inputs: calls in a row, each
with a smaller input than the one before (the last over three label dimensions), bit-exact labels and
energies."""
import numpy as np
import pytest
import torch

from paper_1410_7922_amd import binding as B
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def note(msg):
    print(f"[gpu] {msg}", flush=True)


def test_static_workspace_solve_equals_edp_solve_twice():
    big = synth.workload("stereo384x288")                   # about 60 MB of workspace, near the limit
    small = synth.motion_problem(seed=4, W=72, H=50, r=4)    # 9 x 9 labels, a different tile
    need = B.workspace_size(B.make_problem(torch.from_numpy(big.cost), big.qx, big.qy, big.lam, big.trunc,
                                           big.mode, 1, 50), B.OP_EDP)
    assert need <= (64 << 20) - (4 << 20)
    # then three label dimensions (7 x 7 x 7 labels on the wide tile of four wavefronts per vertex)
    tiny = synth.random_problem(8, 20, 14, 7, 7, 40, 3, 0, 0, 2500, np.int32, qz=7)
    for p, bound in ((big, 50), (small, 2500), (tiny, 2501)):
        note(f"edp_solve_static {p.name}")
        cost = torch.from_numpy(np.ascontiguousarray(p.cost)).to(DEV)
        H, W, _ = p.cost.shape
        lab = torch.full((H, W), -7, dtype=torch.int32, device=DEV)
        en = torch.zeros(1, dtype=torch.int64, device=DEV)
        st = torch.full((1,), 99, dtype=torch.int32, device=DEV)
        B.solve_static(cost, p.qx, p.qy, p.lam, p.trunc, p.mode, 1, cost_bound=bound, labels=lab, energy=en,
                       status=st, qz=p.qz)
        ref_l, ref_e = B.solve(cost, p.qx, p.qy, p.lam, p.trunc, p.mode, 1, cost_bound=bound, qz=p.qz)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert torch.equal(lab, ref_l), p.name
        assert int(en.item()) == int(ref_e.item()), p.name
