#!/usr/bin/env python3
"""Train the learned lag-window proposer for reverberant pairs of 2^18
samples (b = 4, lags [-2^16, 2^16 - 1], 512 bins of 256 lags) and write the
checkpoint and its fallback threshold next to this file.

Everything runs on the GPU: pairs are drawn by the seeded device generator
(synth.config5_reverb_torch), labelled by the library's exact full-range
estimate (the plain method: the bin of its smallest maximising lag), reduced
to the proposer's decimated bf16 input, and the network is trained by the
library's forward, backward and Adam kernels. The threshold on the logit
margin is set on held-out validation pairs (their own seeds): just above the
largest margin of any pair whose top-k bins miss the exact lag, and at least
a given quantile of the margins (a safety share that always takes the full
range).

    python paper_2509_19974_amd/weights/train.py --pairs 1048576 --epochs 2
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N = 1 << 18
LAG = 1 << 16
BITS = 4
NBINS = 512
TRAIN_SALT = 100000      # seeds of the training chunks: TRAIN_SALT + k
VAL_SALT = 50000         # validation: VAL_SALT + k (evaluation sets use salts below 50000)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=1 << 20)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, nargs="+", default=[1e-3, 3e-4])
    ap.add_argument("--val", type=int, default=16384)
    ap.add_argument("--topk", type=int, default=8)
    ap.add_argument("--safety", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=os.path.join(HERE, "proposer_n18"))
    args = ap.parse_args()

    import numpy as np
    import torch
    import synth
    from paper_2509_19974_amd import learned, tde

    assert torch.cuda.is_available(), "training runs on the GPU"
    ctx = tde.Context(0)
    model = tde.Model(ctx, N // 16, NBINS, seed=args.seed)

    def chunks(salt0, total):
        for k in range((total + args.chunk - 1) // args.chunk):
            g = synth.config5_reverb_torch(torch, args.chunk, salt=salt0 + k, n=N, max_lag=LAG)
            yield g["x"], g["y"]

    t0 = time.perf_counter()
    xtr, ltr = learned.make_dataset_device(ctx, model, chunks(TRAIN_SALT, args.pairs), args.pairs, BITS, -LAG,
                                           LAG - 1, log=log)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    log(f"[train] {xtr.shape[0]} training pairs generated and labelled in {gen_s:.1f} s")
    lrs = (args.lr + [args.lr[-1]] * args.epochs)[:args.epochs]
    t1 = time.perf_counter()
    hist = learned.train(ctx, model, xtr, ltr, args.epochs, args.batch, lrs, seed=args.seed, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del xtr, ltr
    log(f"[train] {args.epochs} epochs in {train_s:.1f} s")

    tops, margins, truth = [], [], []
    for x, y in chunks(VAL_SALT, args.val):
        specs = learned.device_specs(x, y, BITS, -LAG, LAG - 1)
        pk = learned.plain_peaks(ctx, specs)
        top, margin = learned.proposals(model, model.prepare(specs), args.topk)
        tops.append(top)
        margins.append(margin)
        truth.append(pk["lag"])
    top, margin, truth = np.concatenate(tops), np.concatenate(margins), np.concatenate(truth)
    theta = learned.tune_threshold(top, margin, truth, NBINS, 0.0, args.safety)
    miss_all, _ = learned.window_misses(top, margin, truth, float("-inf"), NBINS)
    miss_th, fb = learned.window_misses(top, margin, truth, theta, NBINS)
    log(f"[train] validation: {miss_all} of {len(truth)} pairs miss their top-{args.topk} bins; threshold "
        f"{theta:.4f} sends {fb} to the full range and leaves {miss_th} misses")
    model.save(args.out + ".tdem")
    meta = {"n": N, "bits": BITS, "nbins": NBINS, "topk": args.topk, "threshold": theta,
            "train": {"pairs": args.pairs, "epochs": args.epochs, "batch": args.batch, "lr": lrs,
                      "loss_per_epoch": hist, "seed": args.seed, "salts": [TRAIN_SALT, TRAIN_SALT + args.pairs // args.chunk - 1],
                      "generate_and_label_s": gen_s, "train_s": train_s,
                      "train_pairs_per_s": args.pairs * args.epochs / train_s},
            "validation": {"pairs": int(len(truth)), "salts": [VAL_SALT, VAL_SALT + args.val // args.chunk - 1],
                           "misses_before_fallback": miss_all, "fallback": fb, "misses_after_fallback": miss_th,
                           "safety_quantile": args.safety},
            "command": "python paper_2509_19974_amd/weights/train.py " + " ".join(sys.argv[1:])}
    with open(args.out + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
