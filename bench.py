#!/usr/bin/env python3
"""Throughput of the exact integer time-difference estimator on one MI355X.

One step = one call of tde_estimate_batch over the whole batch (Algorithm 1
up to its argmax step for every pair: scale + quantize, exact integer correlation over the
full lag range, argmax), with the float32 inputs already resident in HBM. By
default the call is replayed from its captured HIP graph (use_graph = 1: the
descriptors stay in the workspace, so a step is only kernel launches);
--eager times plain calls (descriptor upload + launches). Stage times (and the
roofline's kernel time) come from an eager pass with the library's stage
events, recorded on the stream the kernels run on.

Default workload: 64 pairs of N = 65536 float32 AR(2) coloured noise (poles
0.95, 0.6), delays uniform in [-N/4, N/4], SNR uniform in [0, 30] dB, uniform
quantizer on [-3 sigma, 3 sigma] with b in {2, 4, 8} (pair i takes b =
(2, 4, 8)[i % 3]), full lag range [-(N-1), N-1].

Prints ONE JSON line (rank 0) with pairs/s, the algorithmic integer MAC rate,
the roofline of the dominant kernel (the int8 matrix-core correlation, timed
with HIP events on the stream it runs on), an FP32 FFT cross-correlation of
the same pairs on the same GPU, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 matrix peak, 5.0 POP/s
FP6_FP4_PEAK_TFLOPS = 10100.0  # MI355X dense FP6 / FP4 matrix peak, 10.1 PFLOP/s
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense bf16 matrix peak, 2.5 PFLOP/s
HBM_PEAK_GBS = 8000.0
# 256 CUs x 16 lanes/clock of 32-bit integer multiply (a quarter of the 64
# lanes/clock of simple VALU ops) x 2.4 GHz, 4 multiplies per Montgomery
# butterfly: 2.46e12 butterflies/s
MODMUL_PEAK_T = 256 * 16 * 2.4e9 / 4 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_macs(nx: int, ny: int, lo: int, hi: int) -> int:
    """sum over tau in [lo, hi] of #{m : 0 <= m < nx, 0 <= m + tau < ny}."""
    import numpy as np
    t = np.arange(lo, hi + 1, dtype=np.int64)
    ov = np.minimum(nx, ny - t) - np.maximum(0, -t)
    return int(np.clip(ov, 0, None).sum())


def make_workload(name: str):
    import synth
    if name == "c2":
        pairs = synth.config2_batch(8, npairs=64, n=65536)
        for i, p in enumerate(pairs):
            p["bits"] = (2, 4, 8)[i % 3]
        desc = {"workload": "batch of 64 pairs, N=65536, AR(2) noise, b in {2,4,8}, full lag range",
                "pairs": 64, "n": 65536, "bits": [2, 4, 8], "lags": "[-(N-1), N-1]"}
        return pairs, desc
    if name == "c1":
        pairs = synth.config1_single(npairs=1)
        desc = {"workload": "single pair, N=4096 white noise, sign quantization, lags [-1024, 1024]",
                "pairs": 1, "n": 4096, "bits": [1], "lags": "[-1024, 1024]"}
        return pairs, desc
    if name.startswith("c3_"):
        lg = int(name[3:])
        n = 1 << lg
        pairs = synth.config3_long(n, npairs=8)
        desc = {"workload": f"8 long pairs, N=2^{lg}, filtered noise, b=8, full lag range", "pairs": 8, "n": n,
                "bits": [8], "lags": "[-(N-1), N-1]"}
        return pairs, desc
    if name == "c4":
        pairs = synth.config4_uneven(4096)
        desc = {"workload": "4096 uneven pairs, N log-uniform in [2^10, 2^18], b in {1,2,4}, lags +-N/4",
                "pairs": 4096, "n": "2^U[10,18]", "bits": [1, 2, 4], "lags": "+-floor(N/4)"}
        return pairs, desc
    if name == "c1x":
        pairs = synth.config1_single(npairs=16384)
        desc = {"workload": "16384 pairs shaped like the single-pair case (N=4096, sign, lags +-1024)",
                "pairs": 16384, "n": 4096, "bits": [1], "lags": "[-1024, 1024]"}
        return pairs, desc
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(kernel_src: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "xcorr_mfma_c2_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != h:
        return None
    return rec.get("hbm_bytes_per_launch")


def fft_baseline(torch, pairs, specs, steps, warmup):
    """FP32 FFT cross-correlation r = irfft(conj(X) Y) of the float signals,
    argmax over each pair's lags (first maximum = smallest lag). Pairs are
    batched by transform length (a power of two covering the pair's lags
    without wrap-around), zero-padded to the longest signal of their batch."""
    groups = {}
    for i, p in enumerate(pairs):
        nx, ny = p["x"].size, p["y"].size
        need = max(p["lag_hi"] + nx, ny - p["lag_lo"])
        nfft = 1
        while nfft < need:
            nfft *= 2
        groups.setdefault(nfft, []).append(i)
    plans = []
    for nfft, idx in groups.items():
        nmax = max(max(pairs[i]["x"].size, pairs[i]["y"].size) for i in idx)
        xs = torch.zeros(len(idx), nmax, device="cuda")
        ys = torch.zeros(len(idx), nmax, device="cuda")
        for k, i in enumerate(idx):
            xs[k, :pairs[i]["x"].size] = specs[i]["x"]
            ys[k, :pairs[i]["y"].size] = specs[i]["y"]
        lo = torch.tensor([pairs[i]["lag_lo"] for i in idx], device="cuda")
        L = max(pairs[i]["lag_hi"] - pairs[i]["lag_lo"] + 1 for i in idx)
        off = torch.arange(L, device="cuda")[None, :]
        valid = off <= torch.tensor([pairs[i]["lag_hi"] - pairs[i]["lag_lo"] for i in idx], device="cuda")[:, None]
        pos = (lo[:, None] + off) % nfft              # circular index of lag tau
        plans.append((nfft, idx, xs, ys, lo, pos, valid))

    def step():
        outs = []
        for nfft, idx, xs, ys, lo, pos, valid in plans:
            X = torch.fft.rfft(xs, n=nfft)
            Y = torch.fft.rfft(ys, n=nfft)
            c = torch.fft.irfft(torch.conj(X) * Y, n=nfft)
            g = torch.gather(c, 1, pos).masked_fill(~valid, float("-inf"))
            outs.append((idx, torch.argmax(g, dim=1) + lo))
        return outs

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        outs = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lag = [0] * len(pairs)
    for idx, l in outs:
        for k, v in zip(idx, l.cpu().numpy().tolist()):
            lag[k] = v
    return ms, lag


def cpu_baseline(pairs, budget_s: float = 12.0):
    """The oracle, pair after pair of the same batch (wrapping round), until
    about budget_s seconds of CPU work are done."""
    import oracle
    t0 = time.perf_counter()
    done = 0
    macs = 0
    while True:
        p = pairs[done % len(pairs)]
        oracle.estimate(p["x"], p["y"], p["bits"], p["lag_lo"], p["lag_hi"])
        done += 1
        macs += alg_macs(p["x"].size, p["y"].size, p["lag_lo"], p["lag_hi"])
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "pairs/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{done} pairs of the {len(pairs)}-pair batch, each Algorithm 1 up to its argmax step "
                      f"(scale, quantize, int64 direct sums over every lag, argmax), {el:.1f} s",
            "int_mac_per_s": macs / el}


def _gen_c5(args_):
    n, npairs, salt = args_
    import synth
    return synth.config5_reverb(npairs=npairs, n=n, max_lag=n // 4, salt=salt)


def run_c5(args):
    """Learned lag-window proposal on reverberant pairs (N = 2^18, b = 4, lags
    [-2^16, 2^16 - 1]): train the proposer on pairs labelled by the exact
    plain estimator, tune the fallback margin on a validation set, then time
    the plain and the learned paths (HIP-graph replays) on 1024 held-out
    pairs and count the lags that differ from the full search."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n = 1 << 18
    chunk = 128
    ntrain, nval, neval = args.c5_train, 512, 1024
    seeds = {"train": [1000 + k for k in range(ntrain // chunk)], "val": [500 + k for k in range(nval // chunk)],
             "eval": list(range(neval // chunk))}
    # generator processes start before anything touches the GPU (or run in
    # this process with --c5-workers 0, e.g. under a profiler)
    pool = None
    if args.c5_workers > 0:
        pool = cf.ProcessPoolExecutor(max_workers=args.c5_workers, mp_context=mp.get_context("spawn"))
        jobs = {k: [pool.submit(_gen_c5, (n, chunk, sd)) for sd in v] for k, v in seeds.items()}
    import numpy as np
    import torch
    from paper_2509_19974_amd import tde, learned
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = tde.Context(0)
    model = tde.Model(ctx, n // 16, 512, seed=1)
    t0 = time.perf_counter()

    def chunks(name):
        for k, sd in enumerate(seeds[name]):
            yield jobs[name][k].result() if pool else _gen_c5((n, chunk, sd))

    xtr, ltr = learned.make_dataset(ctx, model, chunks("train"))
    log(f"[bench] c5 training set ready: {xtr.shape[0]} pairs, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = learned.train(ctx, model, xtr, ltr, args.c5_epochs, 64, args.c5_lr, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del xtr, ltr
    val = [p for c in chunks("val") for p in c]
    vspecs = learned.specs_of(torch, val)
    vtruth = learned.plain_peaks(ctx, vspecs)
    vtop, vmargin = learned.proposals(model, model.prepare(vspecs), 8)
    theta = learned.tune_threshold(vtop, vmargin, vtruth["lag"], 512, 0.0, args.c5_safety)
    del vspecs
    log(f"[bench] c5 threshold {theta:.4f}")
    ev = [p for c in chunks("eval") for p in c]
    if pool:
        pool.shutdown()
    specs = learned.specs_of(torch, ev)
    d = np.array([p["d"] for p in ev])

    def timed(plan):
        ws = torch.empty(plan[2], dtype=torch.uint8, device="cuda")
        out = torch.empty(len(specs) * 24, dtype=torch.uint8, device="cuda")
        for _ in range(max(args.warmup, 1)):
            ctx.estimate_batch(specs, ws=ws, out=out, plan=plan)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.estimate_batch(specs, ws=ws, out=out, plan=plan)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, tde.decode_peaks(out)

    plain_ms, plain = timed(ctx.batch_plan(specs, use_graph=1))
    learn_ms, lrn = timed(ctx.batch_plan(specs, mode=tde.TDE_MODE_LEARNED, model=model, topk=8, margin=theta,
                                         use_graph=1))
    _, lrn0 = timed(ctx.batch_plan(specs, mode=tde.TDE_MODE_LEARNED, model=model, topk=8, margin=-3.0e38,
                                   use_graph=1))

    def differ(a, b):
        return float(np.mean((a["lag"] != b["lag"]) | (a["rmax"] != b["rmax"]) | (a["n_ties"] != b["n_ties"])))

    fallback = float(np.mean((lrn["flags"] & tde.TDE_FLAG_FALLBACK) != 0))
    # stage timing of one eager learned call: CNN + windows (+ fallback) is the engine stage
    tde.tde_timing_read(ctx.handle)
    tde.tde_timing_enable(ctx.handle, True)
    lplan = ctx.batch_plan(specs, mode=tde.TDE_MODE_LEARNED, model=model, topk=8, margin=theta)
    for _ in range(3):
        ctx.estimate_batch(specs, plan=lplan)
    torch.cuda.synchronize()
    stage_ms, stage_n = tde.tde_timing_read(ctx.handle)
    tde.tde_timing_enable(ctx.handle, False)
    engine_ms = stage_ms[1] / max(stage_n[1], 1)
    prop_ms = stage_ms[4] / max(stage_n[4], 1)
    cnn_macs = 2 * (16384 * 32 * 9 + (8192 + 4096 + 2048) * 32 * 32 * 9) + 512 * 1024 * 32
    win_macs = 8 * 256 * n
    result = {
        "metric": "pairs/s and int-MAC/s vs FP32-FFT xcorr on MI355X at oracle-exact lags",
        "value": len(ev) * 1e3 / learn_ms, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": learn_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8+fp6+bf16", "data": "synthetic",
        "config": {"workload": "1024 reverberant pairs, N=2^18, b=4, lags [-2^16, 2^16-1], learned windows (top-8 of "
                               "512 bins, fallback below the tuned margin)", "pairs": len(ev), "n": n},
        "plain": {"pairs_per_s": len(ev) * 1e3 / plain_ms, "ms_per_step": plain_ms},
        "speedup_learned_over_plain": plain_ms / learn_ms,
        "differ_from_full_search": {"before_fallback": differ(lrn0, plain), "after_fallback": differ(lrn, plain)},
        "fallback_fraction": fallback, "threshold": theta,
        "lag_accuracy": {"plain": float(np.mean(plain["lag"] == d)), "learned": float(np.mean(lrn["lag"] == d))},
        "training": {"pairs": ntrain, "epochs": args.c5_epochs, "pairs_per_s": ntrain * args.c5_epochs / train_s,
                     "loss": hist},
        "stage_ms": {"quantize": stage_ms[0] / max(stage_n[0], 1), "engine": engine_ms, "proposer": prop_ms,
                     "argmax": stage_ms[2] / max(stage_n[2], 1)},
        "roofline": {"bound": "mfma", "achieved": 2.0 * cnn_macs * len(ev) / (prop_ms * 1e-3) / 1e12,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": 2.0 * cnn_macs * len(ev) / (prop_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                     "traffic": None, "kernel": "proposer stage: decimated-input CNN forward (bf16 matrix-core "
                                                "convolutions and head, fp32 accumulation) and top-k",
                     "kernel_ms": prop_ms, "alg_cnn_macs_per_pair": cnn_macs, "alg_window_macs_per_pair": win_macs},
    }
    ctx.close()
    print(json.dumps(result), flush=True)


def run_quant(args):
    """Quantizer study: a synthetic analogue of the accuracy-vs-SNR experiment
    of Section 4.2 (speech-like 16000-sample targets delayed by a real
    nu in [0, 64000) inside 80000-sample AR(1) backgrounds). For each SNR:
    the FP32 FFT correlation, and Algorithm 1 without and with its tie-refinement step, with
    the uniform map at b in {1, 2, 4, 8} and the mu-law and Lloyd-Max maps at
    b in {2, 4}. An estimate is correct when every lag of the (refined)
    argmax set is within one sample of nu."""
    import numpy as np
    import torch
    import synth
    from paper_2509_19974_amd import tde
    npairs = args.quant_pairs
    snrs = [-20, -15, -10, -5, 0, 5, 10]
    configs = [(tde.TDE_QUANT_UNIFORM, b) for b in (1, 2, 4, 8)] + \
              [(k, b) for k in (tde.TDE_QUANT_MULAW, tde.TDE_QUANT_GAUSS) for b in (2, 4)]
    names = {tde.TDE_QUANT_UNIFORM: "uniform", tde.TDE_QUANT_MULAW: "mulaw", tde.TDE_QUANT_GAUSS: "gauss"}
    ctx = tde.Context(0)
    lo, hi = 0, 64000
    table = {}
    t_start = time.time()
    for snr in snrs:
        xs, ys, nus = synth.speech_like_mixtures(npairs, float(snr))
        pairs = [dict(x=x, y=y, lag_lo=lo, lag_hi=hi, bits=1) for x, y in zip(xs, ys)]
        base = [dict(x=torch.from_numpy(x).cuda(), y=torch.from_numpy(y).cuda()) for x, y in zip(xs, ys)]
        _, flags = fft_baseline(torch, pairs, base, 1, 0)
        row = {"fft_fp32": float(np.mean(np.abs(np.array(flags) - nus) < 1.0))}
        for kind, bits in configs:
            specs = [dict(x=s["x"], y=s["y"], lag_lo=lo, lag_hi=hi, bits=bits,
                          r_out=torch.empty(hi - lo + 1, dtype=torch.int32, device="cuda"), r_dtype=tde.TDE_I32)
                     for s in base]
            plan = ctx.batch_plan(specs, quantizer=kind)
            out = ctx.estimate_batch(specs, plan=plan)
            torch.cuda.synchronize()
            pk = tde.decode_peaks(out)
            ok4 = ok6 = 0
            for i in range(npairs):
                lag, nt = int(pk[i]["lag"]), int(pk[i]["n_ties"])
                if nt == 1:
                    good = abs(lag - nus[i]) < 1.0
                    ok4 += good
                    ok6 += good
                    continue
                r = specs[i]["r_out"].cpu().numpy()
                tied = np.nonzero(r == r.max())[0] + lo
                ok4 += bool(np.all(np.abs(tied - nus[i]) < 1.0))
                # Algorithm 1, tie-refinement step: the real correlation at the tied lags
                peak = out[24 * i:24 * (i + 1)].clone()
                ctx.refine(specs[i]["x"], specs[i]["y"], specs[i]["r_out"], lo, hi, peak)
                torch.cuda.synchronize()
                rp = tde.decode_peaks(peak)[0]
                if int(rp["n_ties"]) == 1:
                    ok6 += abs(int(rp["lag"]) - nus[i]) < 1.0
                else:      # several lags remain, all among the tied ones: every tied lag must be near nu
                    ok6 += bool(np.all(np.abs(tied - nus[i]) < 1.0))
            key = f"{names[kind]}_b{bits}"
            row[key + "_lines1to4"] = ok4 / npairs
            row[key + "_lines1to6"] = ok6 / npairs
        table[str(snr)] = row
        log(f"[bench] quant snr {snr} dB: " + json.dumps({k: round(v, 3) for k, v in row.items()}))
    result = {
        "metric": "time-difference accuracy vs SNR (share of pairs within one sample)",
        "unit": "fraction", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "quantizer study: 16000-sample speech-like targets, 80000-sample AR(1) backgrounds, "
                               "nu ~ U[0, 64000) with fractional part, lags [0, 64000]",
                   "pairs_per_snr": npairs, "snr_db": snrs},
        "accuracy": table, "seconds": time.time() - t_start,
    }
    ctx.close()
    print(json.dumps(result), flush=True)


def run_refine(args):
    """Tie refinement: when the integer correlation has several maximising
    lags, the real correlation of the unquantized signals decides among them.
    One pair of 65536-sample signals over its full lag range (131071 lags);
    r holds T tied maxima planted within 4096 lags of 0, so each needs a
    float64 dot product over about 65536 samples. A step is one
    tde_refine_ties call (collect the tied lags from r, one dot product per
    tied lag, the refined set), enqueued back to back on one stream; each
    call gets a fresh peak record, since a call rewrites its record."""
    import numpy as np
    import torch
    from paper_2509_19974_amd import tde
    n = 65536
    L = 2 * n - 1
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
    ctx = tde.Context(0)
    lib = tde.load_library()
    stream = torch.cuda.current_stream()
    max_ties = 4096
    wsb = int(lib.tde_refine_workspace_size(max_ties))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    steps, warmup = max(args.steps, 1), args.warmup
    table = {}
    for T in (2, 16, 256):
        r = np.zeros(L, np.int32)
        idx = np.sort(rng.choice(np.arange(n - 1 - 4096, n - 1 + 4096), T, replace=False))
        r[idx] = 1000
        rd = torch.from_numpy(r).cuda()
        rec = np.zeros(1, tde.PEAK_DTYPE)
        rec["lag"], rec["rmax"], rec["n_ties"] = idx[0] - (n - 1), 1000, T
        raw = torch.from_numpy(np.frombuffer(rec.tobytes(), np.uint8).copy())
        peaks = [raw.cuda() for _ in range(steps + warmup)]
        torch.cuda.synchronize()

        def call(pk):
            rc = lib.tde_refine_ties(ctx.handle, x.data_ptr(), n, y.data_ptr(), n, rd.data_ptr(), tde.TDE_I32,
                                     -(n - 1), n - 1, pk.data_ptr(), max_ties, ws.data_ptr(), wsb,
                                     stream.cuda_stream)
            if rc:
                raise tde.TDEError(rc, tde.tde_last_error())

        for k in range(warmup):
            call(peaks[k])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(steps):
            call(peaks[warmup + k])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out = tde.decode_peaks(peaks[-1])[0]
        assert out["flags"] & tde.TDE_FLAG_REFINED and out["n_ties"] >= 1
        table[T] = ms
        log(f"[bench] refine T={T}: {ms * 1e3:.1f} us per call")
    result = {
        "metric": "tie refinements/s (one pair, 65536 samples, full lag range, 16 tied lags)",
        "value": 1e3 / table[16], "unit": "calls/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": table[16], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "refine: N=65536, 131071 lags, tied lags within 4096 of 0", "n": n, "lags": L},
        "us_per_call": {str(T): v * 1e3 for T, v in table.items()},
    }
    print(json.dumps(result), flush=True)


def run_stream(args):
    """Streaming correlation against a template: an 8192-sample template
    buried once in a noisy stream of 64 blocks of 65536 samples, b = 4 codes
    (fixed stream scale); a step is one push. value = stream samples per
    second (each sample makes one lag final, nx MACs)."""
    import numpy as np
    import torch
    from paper_2509_19974_amd import tde
    import synth
    nx, blk, nblk, bits = 8192, 65536, 64, 4
    x, y, where = synth.stream_embedded(nx, blk, nblk)
    yd = torch.from_numpy(y).cuda()
    ctx = tde.Context(0)
    path = {"auto": tde.TDE_PATH_AUTO, "mfma": tde.TDE_PATH_MFMA, "mfma_i8": tde.TDE_PATH_MFMA_I8,
            "popc": tde.TDE_PATH_POPC, "ntt": tde.TDE_PATH_NTT}[args.path]
    sy = (2 * 7 + 1) / (6 * float(np.sqrt(np.mean(y[:blk].astype(np.float64) ** 2))))
    st = tde.Stream(ctx, torch.from_numpy(x).cuda(), bits, sy, blk, path=path)
    stream = torch.cuda.current_stream()
    k = 0
    for _ in range(min(args.warmup, 8)):
        st.push(yd[k * blk:(k + 1) * blk], stream=stream)
        k += 1
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    steps = 0
    while k < nblk:
        _, _, pr = st.push(yd[k * blk:(k + 1) * blk], stream=stream)
        k += 1
        steps += 1
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    _, _, pr = st.finish(stream=stream)
    torch.cuda.synchronize()
    p = tde.decode_peaks(pr)[0]
    fmt = tde.tde_mfma_operand_bits(7, 7, path if path in (tde.TDE_PATH_MFMA, tde.TDE_PATH_MFMA_I8)
                                    else tde.TDE_PATH_MFMA)
    result = {
        "metric": "stream samples/s (lags made final per second) against a template, exact integer correlation",
        "value": blk * 1e3 / ms, "unit": "samples/s", "n_gpus": 1, "steps": steps,
        "warmup": min(args.warmup, 8), "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {4: "fp4", 6: "fp6", 8: "i8"}[fmt], "data": "synthetic",
        "config": {"workload": "stream: 8192-sample template, 64 blocks of 65536 samples, b = 4",
                   "template": nx, "block": blk, "blocks": nblk, "bits": bits},
        "int_mac_per_s": blk * nx * 1e3 / ms,
        "lag_found": int(p["lag"]) == where, "lag": int(p["lag"]), "true_lag": where,
    }
    st.close()
    ctx.close()
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--path", default="auto", choices=["auto", "mfma", "mfma_i8", "popc", "ntt"])
    ap.add_argument("--eager", action="store_true",
                    help="time eager calls instead of HIP-graph replays of the whole call")
    ap.add_argument("--tune", action="store_true", help="run the engine autotuner before planning")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c5-train", type=int, default=8192, help="learned workload: training pairs")
    ap.add_argument("--c5-epochs", type=int, default=4)
    ap.add_argument("--c5-lr", type=float, default=1e-3)
    ap.add_argument("--c5-workers", type=int, default=16)
    ap.add_argument("--c5-safety", type=float, default=0.02,
                    help="learned workload: share of validation margins below the fallback threshold")
    ap.add_argument("--no-fft", action="store_true")
    ap.add_argument("--quant-pairs", type=int, default=256, help="quantizer study: pairs per SNR")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain device copy of this many bytes (scales HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "the pairs of a batch are independent and would be split across GPUs by predicted cost",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "c5":
        run_c5(args)
        return
    if args.workload == "stream":
        run_stream(args)
        return
    if args.workload == "refine":
        run_refine(args)
        return
    if args.workload == "quant":
        run_quant(args)
        return

    import numpy as np
    import torch
    from paper_2509_19974_amd import tde

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"[bench] generating workload {args.workload}")
    pairs, desc = make_workload(args.workload)
    ctx = tde.Context(0)
    specs = [dict(x=torch.from_numpy(p["x"]).cuda(), y=torch.from_numpy(p["y"]).cuda(), lag_lo=p["lag_lo"],
                  lag_hi=p["lag_hi"], bits=p["bits"]) for p in pairs]
    path = {"auto": tde.TDE_PATH_AUTO, "mfma": tde.TDE_PATH_MFMA, "mfma_i8": tde.TDE_PATH_MFMA_I8,
            "popc": tde.TDE_PATH_POPC, "ntt": tde.TDE_PATH_NTT}[args.path]
    if args.tune:
        log("[bench] autotuning engines")
        tde.tde_tune(ctx.handle, 20)
    engines = [tde.tde_tune_query(p["x"].size, p["y"].size, tde.kmax_of_bits(p["bits"]), tde.kmax_of_bits(p["bits"]),
                                  p["lag_lo"], p["lag_hi"]) if path == tde.TDE_PATH_AUTO else path for p in pairs]
    plan = ctx.batch_plan(specs, path=path)
    ws = torch.empty(plan[2], dtype=torch.uint8, device="cuda")
    out = torch.empty(len(pairs) * tde.PEAK_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    macs = sum(alg_macs(p["x"].size, p["y"].size, p["lag_lo"], p["lag_hi"]) for p in pairs)

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.estimate_batch(specs, path, ws=ws, out=out, plan=plan)
    torch.cuda.synchronize()
    tde.tde_timing_read(ctx.handle)
    tde.tde_timing_enable(ctx.handle, True)
    log(f"[bench] timing {args.steps} steps")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.estimate_batch(specs, path, ws=ws, out=out, plan=plan, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    stage_ms, stage_n = tde.tde_timing_read(ctx.handle)
    tde.tde_timing_enable(ctx.handle, False)
    ms_step = total_ms / args.steps
    eager_ms = ms_step
    if not args.eager:
        # the same call replayed from a captured HIP graph (descriptors stay in
        # the workspace); stage timing is not recorded in this mode
        gplan = ctx.batch_plan(specs, path=path, use_graph=1)
        gws = torch.empty(gplan[2], dtype=torch.uint8, device="cuda")
        for _ in range(max(args.warmup, 1)):
            ctx.estimate_batch(specs, path, ws=gws, out=out, plan=gplan, stream=stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            ctx.estimate_batch(specs, path, ws=gws, out=out, plan=gplan, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / args.steps
    pk = tde.decode_peaks(out)
    d = np.array([p["d"] for p in pairs])
    int_correct = float(np.mean((pk["lag"] == d) & (pk["n_ties"] == 1)))
    engine_ms = stage_ms[1] / max(stage_n[1], 1)
    log(f"[bench] {ms_step:.3f} ms/step, engine {engine_ms:.3f} ms, stages {stage_ms} {stage_n}")

    n_ntt = sum(1 for e in engines if e == tde.TDE_PATH_NTT)
    # operand format of every matrix-core pair (codes up to 3: FP4, up to 7:
    # FP6, else int8) and the peak of the mix: MACs over the time each format
    # would take at its own dense peak
    fmt_bits = [tde.tde_mfma_operand_bits(tde.kmax_of_bits(p["bits"]), tde.kmax_of_bits(p["bits"]),
                                          path if path in (tde.TDE_PATH_MFMA, tde.TDE_PATH_MFMA_I8)
                                          else tde.TDE_PATH_MFMA) if e == tde.TDE_PATH_MFMA else 0
                for p, e in zip(pairs, engines)]
    pair_macs = [alg_macs(p["x"].size, p["y"].size, p["lag_lo"], p["lag_hi"]) for p in pairs]
    fmt_names = {4: "fp4", 6: "fp6", 8: "i8"}
    fmt_macs = {fmt_names[f]: sum(m for m, g in zip(pair_macs, fmt_bits) if g == f) for f in (4, 6, 8)}
    dtype = "+".join(k for k in ("fp4", "fp6", "i8") if fmt_macs[k]) or "i8"
    if n_ntt * 2 < len(engines):
        achieved = 2.0 * macs / (engine_ms * 1e-3) / 1e12
        t_at_peak = sum(m / (INT8_PEAK_TOPS if k == "i8" else FP6_FP4_PEAK_TFLOPS) for k, m in fmt_macs.items())
        peak = sum(fmt_macs.values()) / t_at_peak if t_at_peak > 0 else INT8_PEAK_TOPS
        src = os.path.join(ROOT, "paper_2509_19974_amd", "csrc", "k_xcorr_mfma.hip")
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                "frac": achieved / peak, "traffic": traffic_from_profile(src),
                "kernel": "k_xcorr_mfma (32x32 matrix tiles: FP4/FP6 operands with fp32 accumulation for codes "
                          "up to 7, int8 with int32 accumulation beyond)",
                "peak_mix": {k: {"mac_share": m / max(sum(fmt_macs.values()), 1),
                                 "peak": INT8_PEAK_TOPS if k == "i8" else FP6_FP4_PEAK_TFLOPS}
                             for k, m in fmt_macs.items() if m},
                "kernel_ms": engine_ms, "alg_macs_per_launch": macs}
    else:
        # transform engine: modular butterflies (one Montgomery product each)
        # of the three transforms per prime, against the 32-bit multiply rate
        bf = 0
        for p in pairs:
            nx, ny = p["x"].size, p["y"].size
            lo, hi = max(p["lag_lo"], -(nx - 1)), min(p["lag_hi"], ny - 1)
            need = max(hi + nx, ny - lo)
            lg = 13
            while (1 << lg) < need:
                lg += 1
            k = tde.kmax_of_bits(p["bits"])
            nprimes = 1 if min(nx, ny) * k * k < 2013265921 // 2 else 2
            bf += nprimes * 3 * (1 << (lg - 1)) * lg
        achieved = bf / (engine_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": MODMUL_PEAK_T, "unit": "Tbutterfly/s",
                "frac": achieved / MODMUL_PEAK_T, "traffic": None,
                "kernel": "k_ntt_cols_fwd + k_ntt_rows + k_ntt_cols_inv (two-prime NTT, Montgomery)",
                "kernel_ms": engine_ms, "alg_butterflies_per_launch": bf}

    result = {
        "metric": "pairs/s and int-MAC/s vs FP32-FFT xcorr on MI355X at oracle-exact lags",
        "value": len(pairs) * 1e3 / ms_step,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype if n_ntt * 2 < len(engines) else "u32",
        "data": "synthetic",
        "config": desc,
        "int_mac_per_s": macs * 1e3 / ms_step,
        "engines": {name: sum(1 for e in engines if e == code) for name, code in
                    (("mfma", tde.TDE_PATH_MFMA), ("popc", tde.TDE_PATH_POPC), ("ntt", tde.TDE_PATH_NTT))},
        "timing": "eager calls" if args.eager else "hip graph replay",
        "eager_ms_per_step": eager_ms,
        "stage_ms": {"quantize": stage_ms[0] / max(stage_n[0], 1), "engine": engine_ms,
                     "argmax": stage_ms[2] / max(stage_n[2], 1), "call": stage_ms[3] / max(stage_n[3], 1)},
        "lag_accuracy": {"int": int_correct},
        "roofline": roof,
    }
    if not args.no_fft:
        log("[bench] FP32 FFT baseline")
        fms, flag = fft_baseline(torch, pairs, specs, args.steps, args.warmup)
        result["fft_fp32"] = {"pairs_per_s": len(pairs) * 1e3 / fms, "ms_per_step": fms,
                              "lag_accuracy": float(np.mean(np.array(flag) == d)),
                              "speedup_int_over_fft": fms / ms_step}
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(pairs)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
