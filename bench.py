#!/usr/bin/env python3
"""Throughput of the exact integer time-difference estimator on one MI355X.

Default workload, the largest configuration that fits one GPU: 1024
reverberant pairs of N = 2^18 float32 samples (white noise through a random
response with a 60 dB decay over T ~ U[2000, 12000] samples, y = x delayed
by d ~ U{-2^16..2^16-1} plus noise at SNR ~ U[0, 30] dB), the uniform
quantizer on [-3 sigma, 3 sigma] at b = 4, lags [-2^16, 2^16 - 1]. The pairs
are drawn on the GPU by the seeded generator. One step is one
tde_estimate_batch call in learned mode (Algorithm 1 up to its argmax step
with the exact correlation run only where the proposer points): scale and
quantize (with the proposer's decimated input), the trained proposer
(weights committed beside the library), exact correlation inside the top-8
lag bins, the full lag range for pairs whose logit margin is below the
committed threshold, argmax. The float32 inputs are resident in HBM; steps
are replays of the call's captured HIP graph, timed with HIP events on the
stream the kernels run on.

Beside it, on the same pairs: the plain full-range path (the method without
the proposer), an FP32 FFT cross-correlation, the lags that differ from the
full search (on the timed pairs and on 16384 held-out pairs, with 95%
intervals), the CPU oracle on a bounded sample (also the parity check of
the GPU results), stage times from the library's HIP events, and the
roofline of the longest stage. "workloads" holds the other configurations:
the 64 x 65536 batch (mixed b and each b alone), 8 long pairs of 2^22
samples on the transform engine, and 4096 uneven pairs.

Prints ONE JSON line. The exit status is 3 when any GPU result checked
against the oracle differs (the line then says "parity": {"ok": false}).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 matrix peak, 5.0 POP/s
FP6_FP4_PEAK_TFLOPS = 10100.0  # MI355X dense FP6 / FP4 matrix peak, 10.1 PFLOP/s
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense bf16 matrix peak, 2.5 PFLOP/s
HBM_PEAK_GBS = 8000.0
METRIC = "pairs/s and int-MAC/s vs FP32-FFT xcorr on MI355X at oracle-exact lags"
WEIGHTS = os.path.join(ROOT, "paper_2509_19974_amd", "weights", "proposer_n18")
TUNE_TABLE = os.path.join(ROOT, "paper_2509_19974_amd", "weights", "tune_mi355x.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_macs(nx: int, ny: int, lo: int, hi: int) -> int:
    """sum over tau in [lo, hi] of #{m : 0 <= m < nx, 0 <= m + tau < ny}."""
    import numpy as np
    t = np.arange(lo, hi + 1, dtype=np.int64)
    ov = np.minimum(nx, ny - t) - np.maximum(0, -t)
    return int(np.clip(ov, 0, None).sum())


def binom_ci(k: int, n: int):
    """Clopper-Pearson 95% interval of a proportion k/n."""
    from scipy.stats import beta
    lo = 0.0 if k == 0 else float(beta.ppf(0.025, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(0.975, k + 1, n - k))
    return [lo, hi]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def make_workload(name: str):
    import synth
    if name.startswith("c2"):
        pairs = synth.config2_batch(8, npairs=64, n=65536)
        fixed = int(name[4:]) if name.startswith("c2_b") else None
        for i, p in enumerate(pairs):
            p["bits"] = fixed if fixed else (2, 4, 8)[i % 3]
        bits = [fixed] if fixed else [2, 4, 8]
        desc = {"workload": f"batch of 64 pairs, N=65536, AR(2) noise, b in {bits}, full lag range",
                "pairs": 64, "n": 65536, "bits": bits, "lags": "[-(N-1), N-1]"}
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


def stage_traffic(stage: str):
    """HBM bytes per launch of a stage of the learned line, from the committed
    rocprofv3 --pmc summary profiles/learned_c5_pmc.json, if it was taken on
    the stage's current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "learned_c5_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))["stages"][stage]
    except Exception:
        return None
    h = hashlib.sha256(open(os.path.join(ROOT, rec["source"]), "rb").read()).hexdigest()
    return rec["hbm_bytes_per_launch"] if rec.get("source_sha256") == h else None


def traffic_from_profile(kernel_src: str, name: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", name)
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


def fft_baseline(torch, pairs, specs, steps, warmup, stream=None):
    """FP32 FFT cross-correlation r = irfft(conj(X) Y) of the float signals,
    argmax over each pair's lags (first maximum = smallest lag). Pairs are
    batched by transform length (a power of two covering the pair's lags
    without wrap-around), zero-padded to the longest signal of their batch.
    Eager torch calls, timed with events on `stream`."""
    groups = {}
    for i, p in enumerate(pairs):
        nx, ny = p["nx"], p["ny"]
        need = max(p["lag_hi"] + nx, ny - p["lag_lo"])
        nfft = 1
        while nfft < need:
            nfft *= 2
        groups.setdefault(nfft, []).append(i)
    plans = []
    for nfft, idx in groups.items():
        nmax = max(max(pairs[i]["nx"], pairs[i]["ny"]) for i in idx)
        xs = torch.zeros(len(idx), nmax, device="cuda")
        ys = torch.zeros(len(idx), nmax, device="cuda")
        for k, i in enumerate(idx):
            xs[k, :pairs[i]["nx"]] = specs[i]["x"]
            ys[k, :pairs[i]["ny"]] = specs[i]["y"]
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

    stream = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        outs = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lag = [0] * len(pairs)
    for idx, l in outs:
        for k, v in zip(idx, l.cpu().numpy().tolist()):
            lag[k] = v
    del plans
    return ms, lag


def time_batch(ctx, torch, specs, steps, warmup, stream, **plan_kw):
    """Eager calls with the library's stage events, then graph replays of
    the same call. Returns graph and eager ms per step, average stage ms and
    the peaks of the last replay."""
    from paper_2509_19974_amd import tde
    out = torch.empty(len(specs) * tde.PEAK_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    plan = ctx.batch_plan(specs, **plan_kw)
    ws = torch.empty(plan[2], dtype=torch.uint8, device="cuda")
    for _ in range(max(warmup, 1)):
        ctx.estimate_batch(specs, ws=ws, out=out, plan=plan, stream=stream)
    torch.cuda.synchronize()
    tde.tde_timing_read(ctx.handle)
    tde.tde_timing_enable(ctx.handle, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.estimate_batch(specs, ws=ws, out=out, plan=plan, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / steps
    sms, sn = tde.tde_timing_read(ctx.handle)
    tde.tde_timing_enable(ctx.handle, False)
    del ws
    names = ["quantize", "engine", "argmax", "call", "proposer", "windows", "mfma_engine"]
    stage = {names[k]: sms[k] / sn[k] for k in range(len(names)) if sn[k]}
    gplan = ctx.batch_plan(specs, use_graph=1, **plan_kw)
    gws = torch.empty(gplan[2], dtype=torch.uint8, device="cuda")
    for _ in range(max(warmup, 1)):
        ctx.estimate_batch(specs, ws=gws, out=out, plan=gplan, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ctx.estimate_batch(specs, ws=gws, out=out, plan=gplan, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    pk = tde.decode_peaks(out)
    del gws
    return {"graph_ms": graph_ms, "eager_ms": eager_ms, "stage_ms": stage, "peaks": pk}


def mfma_roofline(tde, pairs, engines, path, macs, engine_ms):
    """Roofline of the matrix-core engine: algorithmic ops (2 x sum of
    overlaps) over its launch time, against the peak of its operand-format
    mix (each format's dense peak weighted by its share of the MACs)."""
    fmt_bits = [tde.tde_mfma_operand_bits(tde.kmax_of_bits(p["bits"]), tde.kmax_of_bits(p["bits"]),
                                          path if path in (tde.TDE_PATH_MFMA, tde.TDE_PATH_MFMA_I8)
                                          else tde.TDE_PATH_MFMA) if e == tde.TDE_PATH_MFMA else 0
                for p, e in zip(pairs, engines)]
    pair_macs = [alg_macs(p["nx"], p["ny"], p["lag_lo"], p["lag_hi"]) for p in pairs]
    names = {4: "fp4", 6: "fp6", 8: "i8"}
    fmt_macs = {names[f]: sum(m for m, g in zip(pair_macs, fmt_bits) if g == f) for f in (4, 6, 8)}
    t_at_peak = sum(m / (INT8_PEAK_TOPS if k == "i8" else FP6_FP4_PEAK_TFLOPS) for k, m in fmt_macs.items())
    tot = sum(fmt_macs.values())
    peak = tot / t_at_peak if t_at_peak > 0 else INT8_PEAK_TOPS
    achieved = 2.0 * tot / (engine_ms * 1e-3) / 1e12
    src = os.path.join(ROOT, "paper_2509_19974_amd", "csrc", "k_xcorr_mfma.hip")
    dtype = "+".join(k for k in ("fp4", "fp6", "i8") if fmt_macs[k]) or "i8"
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TOP/s", "frac": achieved / peak,
            "traffic": traffic_from_profile(src, "xcorr_mfma_c2_pmc.json"),
            "kernel": "k_xcorr_mfma (32x32 matrix tiles: FP4/FP6 operands with fp32 accumulation for codes "
                      "up to 7, int8 with int32 accumulation beyond)",
            "peak_mix": {k: {"mac_share": m / max(tot, 1), "peak": INT8_PEAK_TOPS if k == "i8" else FP6_FP4_PEAK_TFLOPS}
                         for k, m in fmt_macs.items() if m},
            "kernel_ms": engine_ms, "alg_macs_per_launch": tot}, dtype


VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9      # 32-bit vector ALU lane operations per second (CUs x SIMDs x lanes x clock)
NTT_BFLY_OPS = 9                            # one lazy Shoup butterfly: mul_hi, 2 mul_lo, sub; add, sub, min; add, sub


def ntt_roofline(tde, pairs, engine_ms, name=""):
    """Roofline of the transform engine. Its kernels are bound by the vector
    ALU: per pair and prime three transforms of n points, (n/2) log2 n
    butterflies each, against the lane-operation rate of the chip divided by
    the nine operations of a lazy butterfly. HBM beside it: per pair and
    prime the three transforms take two passes over their residues (read and
    write, 4 bytes each), 2 x 3 x 2 x 2 x 4 n bytes; one prime when the
    coefficient bound allows it."""
    nbytes, nbfly = 0, 0
    for p in pairs:
        nx, ny = p["nx"], p["ny"]
        lo, hi = max(p["lag_lo"], -(nx - 1)), min(p["lag_hi"], ny - 1)
        need = max(hi + nx, ny - lo)
        lg = 13
        while (1 << lg) < need:
            lg += 1
        k = tde.kmax_of_bits(p["bits"])
        nprimes = 1 if min(nx, ny) * k * k < 998244353 // 2 else 2
        nbytes += nprimes * 3 * 2 * 2 * 4 * (1 << lg)
        nbfly += nprimes * 3 * (1 << (lg - 1)) * lg
    achieved = nbfly / (engine_ms * 1e-3) / 1e9
    peak = VALU_LANE_OPS / NTT_BFLY_OPS / 1e9
    src = os.path.join(ROOT, "paper_2509_19974_amd", "csrc", "k_xcorr_ntt.hip")
    traffic = traffic_from_profile(src, "xcorr_ntt_c3_n22_pmc.json") if name == "c3_22" else None
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "G butterflies/s", "frac": achieved / peak,
            "traffic": traffic, "kernel": "k_ntt_cols_fwd + k_ntt_rows + k_ntt_cols_inv (two-prime NTT)",
            "kernel_ms": engine_ms, "alg_butterflies_per_launch": nbfly,
            "hbm": {"alg_bytes_per_launch": nbytes, "achieved_GBps": nbytes / (engine_ms * 1e-3) / 1e9,
                    "frac": nbytes / (engine_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def run_plain(args, name, path_name="auto", fft=True, cpu_parity=False):
    """One plain (full-search) workload: graph and eager step times, stage
    times, roofline of the correlation engine, FP32 FFT on the same pairs,
    and optionally every pair against the oracle."""
    import numpy as np
    import torch
    from paper_2509_19974_amd import tde
    log(f"[bench] generating workload {name}")
    pairs, desc = make_workload(name)
    for p in pairs:
        p["nx"], p["ny"] = p["x"].size, p["y"].size
    ctx = tde.Context(0)
    stream = torch.cuda.current_stream()
    specs = [dict(x=torch.from_numpy(p["x"]).cuda(), y=torch.from_numpy(p["y"]).cuda(), lag_lo=p["lag_lo"],
                  lag_hi=p["lag_hi"], bits=p["bits"]) for p in pairs]
    path = {"auto": tde.TDE_PATH_AUTO, "mfma": tde.TDE_PATH_MFMA, "mfma_i8": tde.TDE_PATH_MFMA_I8,
            "popc": tde.TDE_PATH_POPC, "ntt": tde.TDE_PATH_NTT}[path_name]
    if args.tune:
        log("[bench] autotuning engines")
        tde.tde_tune(ctx.handle, 20)
    elif args.tune_table:
        log(f"[bench] engine table {args.tune_table}")
        tde.tde_tune_load(args.tune_table)
    engines = [tde.tde_tune_query(p["nx"], p["ny"], tde.kmax_of_bits(p["bits"]), tde.kmax_of_bits(p["bits"]),
                                  p["lag_lo"], p["lag_hi"]) if path == tde.TDE_PATH_AUTO else path for p in pairs]
    macs = sum(alg_macs(p["nx"], p["ny"], p["lag_lo"], p["lag_hi"]) for p in pairs)
    log(f"[bench] {name}: timing {args.steps} steps")
    t = time_batch(ctx, torch, specs, args.steps, args.warmup, stream, path=path)
    ms_step = t["eager_ms"] if args.eager else t["graph_ms"]
    pk = t["peaks"]
    d = np.array([p["d"] for p in pairs])
    n_ntt = sum(1 for e in engines if e == tde.TDE_PATH_NTT)
    if n_ntt * 2 < len(engines):
        roof, dtype = mfma_roofline(tde, pairs, engines, path, macs, t["stage_ms"].get("mfma_engine", t["stage_ms"]["engine"]))
    else:
        roof, dtype = ntt_roofline(tde, pairs, t["stage_ms"]["engine"], name), "u32"
    res = {"pairs_per_s": len(pairs) * 1e3 / ms_step, "ms_per_step": ms_step, "timing": "eager calls" if args.eager
           else "hip graph replay", "eager_ms_per_step": t["eager_ms"], "int_mac_per_s": macs * 1e3 / ms_step,
           "dtype": dtype, "config": desc,
           "engines": {nm: sum(1 for e in engines if e == code) for nm, code in
                       (("mfma", tde.TDE_PATH_MFMA), ("popc", tde.TDE_PATH_POPC), ("ntt", tde.TDE_PATH_NTT))},
           "stage_ms": t["stage_ms"], "lag_accuracy": {"int": float(np.mean((pk["lag"] == d) & (pk["n_ties"] == 1)))},
           "roofline": roof}
    if fft:
        fms, flag = fft_baseline(torch, pairs, specs, args.steps, args.warmup, stream)
        res["fft_fp32"] = {"pairs_per_s": len(pairs) * 1e3 / fms, "ms_per_step": fms,
                           "lag_accuracy": float(np.mean(np.array(flag) == d)),
                           "speedup_int_graph_over_fft": fms / t["graph_ms"],
                           "speedup_int_eager_over_fft": fms / t["eager_ms"]}
    if n_ntt * 2 >= len(engines) and name.startswith("c3_"):
        res["direct_mfma_1_64"] = direct_mfma_slice(tde, ctx, torch, specs, pairs, args, t)
    if cpu_parity:
        import oracle
        t0 = time.perf_counter()
        bad = 0
        for i, p in enumerate(pairs):
            ref = oracle.estimate(p["x"], p["y"], p["bits"], p["lag_lo"], p["lag_hi"])
            bad += (int(pk[i]["lag"]), int(pk[i]["rmax"]), int(pk[i]["n_ties"])) != \
                   (ref["lag"], ref["rmax"], ref["n_ties"])
        res["parity"] = {"oracle_pairs": len(pairs), "mismatches": bad, "ok": bad == 0,
                         "oracle_s": time.perf_counter() - t0}
    ctx.close()
    del specs
    torch.cuda.empty_cache()
    return res


def direct_mfma_slice(tde, ctx, torch, specs, pairs, args, t_ntt):
    """The long-signal pairs on the direct matrix-core engine over the central
    1/64 of their lags, beside the transform engine over all of them: both
    engines' r over that slice compared bit for bit, the direct engine's
    time on the slice, and that time scaled to the full range by MACs."""
    sl, full_macs, part_macs = [], 0, 0
    for s, p in zip(specs, pairs):
        L = (p["lag_hi"] - p["lag_lo"] + 1 + 63) // 64
        lo = -(L // 2)
        sl.append(dict(s, lag_lo=lo, lag_hi=lo + L - 1))
        full_macs += alg_macs(p["nx"], p["ny"], p["lag_lo"], p["lag_hi"])
        part_macs += alg_macs(p["nx"], p["ny"], lo, lo + L - 1)
    t = time_batch(ctx, torch, sl, args.steps, args.warmup, torch.cuda.current_stream(), path=tde.TDE_PATH_MFMA)
    # r over the slice from both engines (one eager call each, outside the timing)
    same = True
    for s in sl:
        n = s["lag_hi"] - s["lag_lo"] + 1
        rs = []
        for path in (tde.TDE_PATH_NTT, tde.TDE_PATH_MFMA):
            r = torch.empty(n, dtype=torch.int64, device="cuda")
            ctx.estimate_batch([dict(s, r_out=r, r_dtype=tde.TDE_I64)], path=path)
            rs.append(r)
        torch.cuda.synchronize()
        same = same and bool(torch.equal(rs[0], rs[1]))
        del rs
    ms = t["graph_ms"]
    return {"lags": "central 1/64 of each pair's range", "ms_per_step": ms, "pairs_per_s": len(sl) * 1e3 / ms,
            "int_mac_per_s": part_macs * 1e3 / ms, "mac_share_of_full_range": part_macs / full_macs,
            "full_range_ms_scaled_by_macs": ms * full_macs / part_macs,
            "transform_engine_full_range_ms": t_ntt["graph_ms"],
            "transform_speedup_over_direct_scaled": ms * full_macs / part_macs / t_ntt["graph_ms"],
            "r_equal_to_transform_engine": same}


def window_macs(top, fallback, n, nbins, bin_lags=256):
    """Exact MACs the learned step computes: for a pair on its windows, the
    overlaps of every lag in its top bins; for a fallback pair, the full range."""
    import numpy as np
    half = nbins // 2
    full = alg_macs(n, n, -half * bin_lags, half * bin_lags - 1)
    tot = 0
    for k in range(top.shape[0]):
        if fallback[k]:
            tot += full
            continue
        for b in top[k]:
            lo = (int(b) - half) * bin_lags
            t = np.arange(lo, lo + bin_lags)
            tot += int(np.clip(n - np.abs(t), 0, None).sum())
    return tot


def run_c5(args):
    """The default line (see the module docstring)."""
    import numpy as np
    import torch
    import synth
    import oracle
    from paper_2509_19974_amd import learned, tde
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n, lag, bits, nbins, npairs = 1 << 18, 1 << 16, 4, 512, 1024
    meta = json.load(open(WEIGHTS + ".json"))
    theta, topk = float(meta["threshold"]), int(meta["topk"])
    ctx = tde.Context(0)
    stream = torch.cuda.current_stream()
    model = tde.Model(ctx, n // 16, nbins)
    model.load(WEIGHTS + ".tdem")
    if args.tune_table:
        tde.tde_tune_load(args.tune_table)
    log("[bench] generating 1024 reverberant pairs on the GPU")
    g = [synth.config5_reverb_torch(torch, 512, salt=s, n=n, max_lag=lag) for s in (0, 1)]
    X = torch.cat([a["x"] for a in g])
    Y = torch.cat([a["y"] for a in g])
    d = torch.cat([a["d"] for a in g]).cpu().numpy()
    del g
    specs = learned.device_specs(X, Y, bits, -lag, lag - 1)
    pairs = [dict(nx=n, ny=n, lag_lo=-lag, lag_hi=lag - 1, bits=bits) for _ in range(npairs)]

    log("[bench] c5: plain full-range path")
    tp = time_batch(ctx, torch, specs, args.steps, args.warmup, stream)
    log("[bench] c5: learned path")
    tl = time_batch(ctx, torch, specs, args.steps, args.warmup, stream, mode=tde.TDE_MODE_LEARNED, model=model,
                    topk=topk, margin=theta)
    t0 = time_batch(ctx, torch, specs, 1, 1, stream, mode=tde.TDE_MODE_LEARNED, model=model, topk=topk,
                    margin=float("-inf"))
    plain, lrn, lrn0 = tp["peaks"], tl["peaks"], t0["peaks"]

    def differ(a, b):
        return int(np.count_nonzero((a["lag"] != b["lag"]) | (a["rmax"] != b["rmax"]) | (a["n_ties"] != b["n_ties"])))

    fb_mask = (lrn["flags"] & tde.TDE_FLAG_FALLBACK) != 0
    _, top, _ = model.forward(model.prepare(specs), topk=topk)
    win_macs = window_macs(top.cpu().numpy(), fb_mask, n, nbins)
    full_macs = npairs * alg_macs(n, n, -lag, lag - 1)

    log("[bench] c5: held-out pairs for the differ rates")
    held = {"pairs": 0, "before": 0, "after": 0, "fallback": 0}
    for s in range(10, 10 + args.c5_heldout // 1024):
        gg = [synth.config5_reverb_torch(torch, 512, salt=2 * s + h, n=n, max_lag=lag) for h in (0, 1)]
        hs = learned.device_specs(torch.cat([a["x"] for a in gg]), torch.cat([a["y"] for a in gg]), bits, -lag,
                                  lag - 1)
        a = tde.decode_peaks(ctx.estimate_batch(hs))
        b = tde.decode_peaks(ctx.estimate_batch(hs, plan=ctx.batch_plan(
            hs, mode=tde.TDE_MODE_LEARNED, model=model, topk=topk, margin=theta)))
        c = tde.decode_peaks(ctx.estimate_batch(hs, plan=ctx.batch_plan(
            hs, mode=tde.TDE_MODE_LEARNED, model=model, topk=topk, margin=float("-inf"))))
        held["pairs"] += len(hs)
        held["before"] += differ(c, a)
        held["after"] += differ(b, a)
        held["fallback"] += int(np.count_nonzero(b["flags"] & tde.TDE_FLAG_FALLBACK))
        del hs, gg
    torch.cuda.synchronize()

    log("[bench] c5: FP32 FFT baseline")
    fspecs = [dict(x=X[i], y=Y[i]) for i in range(npairs)]
    fms, flag = fft_baseline(torch, pairs, fspecs, max(args.steps // 4, 2), 1, stream)
    torch.cuda.empty_cache()

    st_l, st_p = tl["stage_ms"], tp["stage_ms"]
    # per-stage rooflines of the learned step
    samples = 2 * npairs * n
    cnn_macs = 2 * (16384 * 32 * 9 + (8192 + 4096 + 2048) * 32 * 32 * 9) + nbins * 1024 * 32
    roofs = {}
    qb = samples * (4 + 1 + 0.125)        # float in, int8 code out, bf16 decimated value per 16 samples
    roofs["quantize"] = {"bound": "hbm", "achieved": qb / (st_l["quantize"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "kernel": "k_sumsq_blocks + k_quantize (scale, codes, decimated input)",
                         "kernel_ms": st_l["quantize"], "alg_bytes_per_launch": qb}
    roofs["proposer"] = {"bound": "mfma", "achieved": 2.0 * cnn_macs * npairs / (st_l["proposer"] * 1e-3) / 1e12,
                         "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "kernel": "CNN forward (bf16 matrix-core convolutions, head) and top-k",
                         "kernel_ms": st_l["proposer"], "alg_macs_per_launch": cnn_macs * npairs}
    wm = window_macs(top.cpu().numpy(), np.zeros(npairs, bool), n, nbins)
    roofs["windows"] = {"bound": "mfma", "achieved": 2.0 * wm / (st_l["windows"] * 1e-3) / 1e12,
                        "peak": FP6_FP4_PEAK_TFLOPS, "unit": "TFLOP/s", "kernel": "k_xcorr_win_fp<6> (exact "
                        "correlation in the top-8 bins, FP6 matrix operands, one 32-row tile per pair)",
                        "kernel_ms": st_l["windows"], "alg_macs_per_launch": wm}
    if "mfma_engine" in st_l:
        fm = int(np.count_nonzero(fb_mask)) * alg_macs(n, n, -lag, lag - 1)
        roofs["fallback"] = {"bound": "mfma", "achieved": 2.0 * fm / (st_l["mfma_engine"] * 1e-3) / 1e12,
                             "peak": FP6_FP4_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "kernel": "k_xcorr_mfma over the fallback pairs (FP6 operands)",
                             "kernel_ms": st_l["mfma_engine"], "alg_macs_per_launch": fm}
    for st, r in roofs.items():
        r["frac"] = r["achieved"] / r["peak"]
        r["traffic"] = stage_traffic(st)
    dom = max(roofs, key=lambda k: roofs[k]["kernel_ms"])
    roof = dict(roofs[dom], stage=dom)

    log("[bench] c5: CPU oracle (baseline and parity sample)")
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        Xh, Yh = X.cpu().numpy(), Y.cpu().numpy()
        t_start = time.perf_counter()
        bad_plain = bad_learned = 0
        done = 0
        while done < npairs:
            ref = oracle.estimate(Xh[done], Yh[done], bits, -lag, lag - 1)
            got = (ref["lag"], ref["rmax"], ref["n_ties"])
            bad_plain += (int(plain[done]["lag"]), int(plain[done]["rmax"]), int(plain[done]["n_ties"])) != got
            bad_learned += (int(lrn[done]["lag"]), int(lrn[done]["rmax"]), int(lrn[done]["n_ties"])) != got
            done += 1
            if time.perf_counter() - t_start > args.cpu_budget:
                break
        el = time.perf_counter() - t_start
        threads = oracle.threads()
        # one thread, on a lag subset of one pair (linear in MACs)
        oracle.set_threads(1)
        sub_lo, sub_hi = -2048, 2047
        t1 = time.perf_counter()
        oracle.xcorr(oracle.quantize(Xh[0], bits)[0], oracle.quantize(Yh[0], bits)[0], sub_lo, sub_hi)
        el1 = time.perf_counter() - t1
        oracle.set_threads(threads)
        sub_macs = alg_macs(n, n, sub_lo, sub_hi)
        pair_macs = alg_macs(n, n, -lag, lag - 1)
        cpu = {"value": done / el, "unit": "pairs/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{done} of the 1024 timed pairs, each Algorithm 1 up to its argmax step (scale, quantize, "
                         f"int64 direct sums over all 131072 lags, argmax), {el:.1f} s on {threads} threads",
               "int_mac_per_s": done * pair_macs / el,
               "single_thread": {"pairs_per_s": sub_macs / el1 / pair_macs, "int_mac_per_s": sub_macs / el1,
                                 "sample": f"int64 direct sums of one pair over lags [{sub_lo}, {sub_hi}] "
                                           f"({sub_macs} MACs, {el1:.2f} s), extrapolated linearly in MACs"}}
        parity = {"oracle_pairs": done, "plain_mismatches": bad_plain, "learned_mismatches": bad_learned,
                  "ok": bad_plain == 0 and bad_learned == 0,
                  "check": "(lag, rmax, n_ties) of the plain and the learned GPU results against the oracle"}

    lms = tl["eager_ms"] if args.eager else tl["graph_ms"]
    pms = tp["eager_ms"] if args.eager else tp["graph_ms"]
    hp = held["pairs"]
    result = {
        "metric": METRIC, "value": npairs * 1e3 / lms, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": lms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8+bf16+fp6", "data": "synthetic",
        "config": {"workload": "1024 reverberant pairs, N=2^18, b=4, lags [-2^16, 2^16-1], learned windows "
                               "(top-8 of 512 bins, full-range fallback below the margin threshold)",
                   "pairs": npairs, "n": n, "bits": bits, "topk": topk, "threshold": theta,
                   "proposer": "paper_2509_19974_amd/weights/proposer_n18.tdem"},
        "timing": "eager calls" if args.eager else "hip graph replay",
        "eager_ms_per_step": tl["eager_ms"],
        "int_mac_per_s": win_macs * 1e3 / lms,
        "full_range_equivalent_mac_per_s": full_macs * 1e3 / lms,
        "plain": {"pairs_per_s": npairs * 1e3 / pms, "ms_per_step": pms, "eager_ms_per_step": tp["eager_ms"],
                  "int_mac_per_s": full_macs * 1e3 / pms, "stage_ms": st_p,
                  "roofline": mfma_roofline(tde, pairs, [tde.TDE_PATH_MFMA] * npairs, tde.TDE_PATH_AUTO, full_macs,
                                            st_p.get("mfma_engine", st_p["engine"]))[0]},
        "speedup_learned_over_plain": pms / lms,
        "differ_from_full_search": {
            "timed_pairs": {"pairs": npairs, "before_fallback": differ(lrn0, plain),
                            "after_fallback": differ(lrn, plain)},
            "held_out": {"pairs": hp, "before_fallback": held["before"],
                         "before_fallback_rate": held["before"] / max(hp, 1),
                         "before_fallback_ci95": binom_ci(held["before"], hp) if hp else None,
                         "after_fallback": held["after"], "after_fallback_rate": held["after"] / max(hp, 1),
                         "after_fallback_ci95": binom_ci(held["after"], hp) if hp else None,
                         "fallback_fraction": held["fallback"] / max(hp, 1)}},
        "fallback_fraction": float(np.mean(fb_mask)),
        "lag_accuracy": {"plain": float(np.mean(plain["lag"] == d)), "learned": float(np.mean(lrn["lag"] == d)),
                         "fft_fp32": float(np.mean(np.array(flag) == d))},
        "stage_ms": st_l,
        "fft_fp32": {"pairs_per_s": npairs * 1e3 / fms, "ms_per_step": fms, "timing": "eager torch calls",
                     "speedup_learned_graph_over_fft": fms / tl["graph_ms"],
                     "speedup_learned_eager_over_fft": fms / tl["eager_ms"],
                     "speedup_plain_graph_over_fft": fms / tp["graph_ms"],
                     "speedup_plain_eager_over_fft": fms / tp["eager_ms"]},
        "roofline": roof, "roofline_stages": roofs,
        "training": meta["train"],
    }
    if cpu:
        result["cpu_baseline"] = cpu
        result["parity"] = parity
    model.close()
    ctx.close()
    del X, Y, specs
    torch.cuda.empty_cache()
    return result


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
        pairs = [dict(x=x, y=y, nx=x.size, ny=y.size, lag_lo=lo, lag_hi=hi, bits=1) for x, y in zip(xs, ys)]
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
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--path", default="auto", choices=["auto", "mfma", "mfma_i8", "popc", "ntt"])
    ap.add_argument("--eager", action="store_true",
                    help="time eager calls instead of HIP-graph replays of the whole call")
    ap.add_argument("--tune", action="store_true", help="run the engine autotuner before planning")
    ap.add_argument("--tune-table", default=TUNE_TABLE,
                    help="engine and tile-width table measured on MI355X ('' for the built-in rules)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-workloads", action="store_true", help="default line only, without the other configs")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of CPU oracle work")
    ap.add_argument("--c5-heldout", type=int, default=16384, help="held-out pairs for the differ rates")
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
    special = {"stream": run_stream, "refine": run_refine, "quant": run_quant}
    if args.workload in special:
        special[args.workload](args)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "c5":
        result = run_c5(args)
        if not args.no_workloads:
            wl = {}
            wl["c2"] = run_plain(args, "c2", cpu_parity=not args.no_cpu_baseline)
            for b in (2, 4, 8):
                wl[f"c2_b{b}"] = run_plain(args, f"c2_b{b}", fft=False)
            wl["c3_22"] = run_plain(args, "c3_22", path_name="ntt")
            wl["c4"] = run_plain(args, "c4")
            result["workloads"] = wl
        ok = all(r.get("parity", {}).get("ok", True) for r in [result] + list(result.get("workloads", {}).values()))
    else:
        res = run_plain(args, args.workload, args.path, fft=not args.no_fft, cpu_parity=not args.no_cpu_baseline)
        result = {"metric": METRIC, "value": res.pop("pairs_per_s"), "unit": "pairs/s", "n_gpus": 1,
                  "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
                  "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": res.pop("dtype"),
                  "data": "synthetic", "config": res.pop("config")}
        result.update(res)
        ok = result.get("parity", {}).get("ok", True)
    print(json.dumps(result), flush=True)
    if not ok:
        log("[bench] PARITY FAILURE: a GPU result differs from the oracle")
        sys.exit(3)


if __name__ == "__main__":
    main()
