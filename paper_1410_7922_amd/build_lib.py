"""Build ``libedp.so`` (the gfx950 HIP library behind include/edp.h) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libedp.so")
SOURCES = [
    # scan and marginal kernels: linear RMS (t*) and general RMS window kinds (q*) per tile group
    "edp_pass_t0.hip", "edp_pass_t1.hip", "edp_pass_t2.hip", "edp_pass_t3.hip",
    "edp_pass_q0.hip", "edp_pass_q1.hip", "edp_pass_q2.hip", "edp_pass_q3.hip",
    "edp_api.hip", "edp_pass.hip",
    # scans and marginal of the wide-vertex tiles (a vertex on several wavefronts)
    "edp_pass_mv.hip",
    # scans and marginal of the tiles of three-dimensional label spaces
    "edp_pass_z.hip",
    # edp_solve with its workspace in a static device array (callers that cannot allocate)
    "edp_static.hip",
    # scanline DP: choice indexes and backtracking; min-marginals per tile group
    "edp_dp.hip", "edp_dpm.hip", "edp_dpm_a.hip", "edp_dpm_b.hip", "edp_dpm_c.hip",
    "edp_misc.hip", "edp_cnn.hip", "edp_learn_api.hip",
]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link the shared library; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    objs = []
    failed = []
    for src, obj, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
        objs.append(obj)
    if failed:
        msg = "\n".join(f"--- {s} ---\n{t}" for s, t in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
