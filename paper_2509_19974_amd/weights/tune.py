#!/usr/bin/env python3
"""Measure the engine and tile-width tuning table on this GPU (tde_tune) and
write it next to this file, for tde_tune_load.

    python paper_2509_19974_amd/weights/tune.py --max-log-n 20
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-log-n", type=int, default=20)
    ap.add_argument("--out", default=os.path.join(HERE, "tune_mi355x.txt"))
    args = ap.parse_args()
    import torch
    from paper_2509_19974_amd import tde
    assert torch.cuda.is_available(), "tuning runs on the GPU"
    ctx = tde.Context(0)
    t0 = time.perf_counter()
    tde.tde_tune(ctx.handle, args.max_log_n)
    tde.tde_tune_save(args.out)
    print(f"tuning table for sizes 2^10 .. 2^{args.max_log_n} written to {args.out} "
          f"in {time.perf_counter() - t0:.1f} s", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
