"""Train the label-window network on the GPU with the library's own kernels.

Training pairs: synthetic two-frame motion instances (31 x 31 labels, squared
difference cost truncated at 2500, lambda 15, T 3 per dimension), each solved
by the plain EDP (j = 1) on the GPU; the network learns the plain labels from
the pooled cost volume.  Frames come from the seeded generator (CPU worker
processes, started before the GPU is touched); the cost volume, the plain
solve, pooling, the network and Adam run on the GPU.

  python -m paper_1410_7922_amd.train_window --instances 10000 --size 320x240 \\
      --out paper_1410_7922_amd/weights/window_net_31x31.npz

Prints one progress line per stage and writes a JSON log next to the weights.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

R = 15          # label range +-15: 31 x 31 labels
CMAX = 2500
SCALE = 250     # network input normaliser
LAM, TRUNC = 15, 3


def _frames(args):
    import synth
    seed, W, H = args
    i0, i1, _, _ = synth.motion_frames(seed=seed, W=W, H=H, r=R)
    return i0, i1


def make_frames(seeds, W, H, workers):
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_frames, [(s, W, H) for s in seeds], chunksize=16)


def log(msg):
    print(f"[train] {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=10000)
    ap.add_argument("--size", default="320x240")
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--val", type=int, default=64, help="held-out instances (seeds after the training ones)")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--decay", type=float, default=0.7, help="learning-rate factor per epoch")
    ap.add_argument("--loss-window", type=int, default=1, help="window of the training loss (1: cross entropy)")
    ap.add_argument("--pool-mode", type=int, default=1, help="network input: 0 label blocks, 1 label rows/columns")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_1410_7922_amd", "weights", "window_net_31x31.npz"))
    args = ap.parse_args()
    W, H = (int(v) for v in args.size.split("x"))

    t0 = time.time()
    seeds = list(range(args.seed0, args.seed0 + args.instances + args.val))
    frames = make_frames(seeds, W, H, args.workers)          # before the GPU is touched
    log(f"{len(frames)} frame pairs {W}x{H} generated in {time.time() - t0:.1f} s")

    import torch

    import paper_1410_7922_amd as edp
    from paper_1410_7922_amd import binding as B
    from paper_1410_7922_amd.learned import window_hit_rate
    from paper_1410_7922_amd.window import WindowNet

    dev = torch.device("cuda:0")
    n = len(frames)
    h, w = H // 2, W // 2
    X = torch.empty((n, h, w, 64), dtype=torch.int16, device=dev)
    TX = torch.empty((n, h * w), dtype=torch.int32, device=dev)
    TY = torch.empty((n, h * w), dtype=torch.int32, device=dev)
    labels_val = []
    cost = torch.empty((H, W, (2 * R + 1) ** 2), dtype=torch.int32, device=dev)
    ws = edp.Workspace()
    lab = torch.empty((H, W), dtype=torch.int32, device=dev)
    en = torch.empty(1, dtype=torch.int64, device=dev)
    net = WindowNet(dev, seed=args.init_seed, pool_mode=args.pool_mode)
    t1 = time.time()
    for k, (i0, i1) in enumerate(frames):
        B.dsi_motion(torch.from_numpy(i0).to(dev), torch.from_numpy(i1).to(dev), R, CMAX, out=cost)
        edp.solve(cost, 2 * R + 1, 2 * R + 1, LAM, TRUNC, 0, 1, cost_bound=CMAX, ws=ws, labels=lab, energy=en)
        B.pool_cost(cost, 2 * R + 1, 2 * R + 1, SCALE, out=X[k], mode=args.pool_mode)
        tx, ty = net.targets(lab, 2 * R + 1)
        TX[k].copy_(tx)
        TY[k].copy_(ty)
        if k >= args.instances:
            labels_val.append(lab.clone())
        if (k + 1) % 1000 == 0:
            torch.cuda.synchronize()
            log(f"labelled {k + 1}/{n} instances with the plain EDP ({time.time() - t1:.1f} s)")
    torch.cuda.synchronize()
    label_s = time.time() - t1
    del cost, ws
    torch.cuda.empty_cache()

    def validate():
        hits, losses = [], []
        for j in range(args.val):
            k = args.instances + j
            logits = net.forward(X[k])
            net.backward(X[k], TX[k], TY[k], args.loss_window)
            losses.append(float(net.loss.item()))
            cen = torch.empty((H, W, 2), dtype=torch.int32, device=dev)
            B.decode_windows(logits, h, w, 64, 2 * R + 1, 2 * R + 1, 7, 31, cen)
            hits.append(window_hit_rate(cen, labels_val[j], 2 * R + 1, 7))
        return float(np.mean(losses)), float(np.mean(hits))

    history = []
    rng = np.random.default_rng(args.init_seed)
    steps = 0
    t2 = time.time()
    for ep in range(args.epochs):
        order = rng.permutation(args.instances)
        lr = args.lr * (args.decay ** ep)
        tot = torch.zeros(1, dtype=torch.float32, device=dev)
        for k in order:
            loss = net.train_step(X[k], TX[k], TY[k], lr, args.loss_window)
            tot += loss
            steps += 1
        vl, vh = validate()
        history.append({"epoch": ep + 1, "lr": lr, "train_loss": float(tot.item()) / args.instances,
                        "val_loss": vl, "val_window_hit_rate": vh, "seconds": time.time() - t2})
        log(f"epoch {ep + 1}: train loss {history[-1]['train_loss']:.4f}, val loss {vl:.4f}, "
            f"val window hit rate {vh:.4f} ({time.time() - t2:.1f} s)")
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    meta = {"instances": args.instances, "size": [W, H], "seed0": args.seed0, "val": args.val,
            "epochs": args.epochs, "lr": args.lr, "decay": args.decay, "loss_window": args.loss_window, "pool_mode": args.pool_mode, "input_scale": SCALE, "steps": steps, "labelling_seconds": label_s,
            "training_seconds": time.time() - t2, "history": history,
            "problem": {"labels": [2 * R + 1, 2 * R + 1], "cmax": CMAX, "lambda": LAM, "trunc": TRUNC,
                        "mode": "per-dimension", "iterations": 1}}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"weights written to {args.out}")


if __name__ == "__main__":
    main()
