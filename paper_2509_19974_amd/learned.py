"""Training and evaluation helpers for the learned lag-window proposer.

The proposer (tde_model) only decides where the exact correlation
(the correlation step of Algorithm 1) runs; its labels come from the plain method itself: the
exact full-range argmax of the integer correlation, mapped to the 256-lag
bin that holds it. Everything numeric runs in libtde (quantize, exact
correlation, the CNN's forward/backward/Adam); this module only sequences the
calls and keeps arrays in device memory through PyTorch.
"""
from __future__ import annotations

import numpy as np

from . import tde

BIN = 256          # raw lags per bin (16x decimation, then 4 poolings of 2)


def bins_of_lags(lags, nbins: int) -> np.ndarray:
    return np.clip((np.asarray(lags, np.int64) + (nbins // 2) * BIN) // BIN, 0, nbins - 1).astype(np.int32)


def specs_of(torch, pairs, device="cuda"):
    return [dict(x=torch.from_numpy(p["x"]).to(device), y=torch.from_numpy(p["y"]).to(device),
                 lag_lo=p["lag_lo"], lag_hi=p["lag_hi"], bits=p["bits"]) for p in pairs]


def plain_peaks(ctx, specs, use_graph=0):
    """Exact full-range estimate of every pair (the method without the
    proposer); returns the decoded peaks."""
    out = ctx.estimate_batch(specs, tde.TDE_PATH_AUTO) if not use_graph else None
    return tde.decode_peaks(out)


def learned_peaks(ctx, specs, model, topk: int, theta: float):
    plan = ctx.batch_plan(specs, mode=tde.TDE_MODE_LEARNED, model=model, topk=topk, margin=theta)
    return tde.decode_peaks(ctx.estimate_batch(specs, plan=plan))


def make_dataset(ctx, model, pair_chunks, log=None):
    """Inputs (bf16 decimated pairs, device) and labels (bins of the exact
    lags, device int32) for chunks of pairs given as lists of dicts."""
    torch = ctx.torch
    xs, ls = [], []
    for k, pairs in enumerate(pair_chunks):
        specs = specs_of(torch, pairs)
        pk = plain_peaks(ctx, specs)
        xs.append(model.prepare(specs))
        ls.append(torch.from_numpy(bins_of_lags(pk["lag"], model.nbins)).cuda())
        if log:
            log(f"[learned] dataset chunk {k}: {len(pairs)} pairs")
    return torch.cat(xs), torch.cat(ls)


def device_specs(x, y, bits: int, lag_lo: int, lag_hi: int):
    """Batch specs for the rows of two device tensors [B][n] (one pair per row)."""
    return [dict(x=x[i], y=y[i], lag_lo=lag_lo, lag_hi=lag_hi, bits=bits) for i in range(x.shape[0])]


def make_dataset_device(ctx, model, chunks, npairs: int, bits: int, lag_lo: int, lag_hi: int, log=None):
    """Training set generated and labelled on the device: `chunks` yields
    (x, y) device tensors [B][n]; each chunk is labelled by the exact
    full-range plain estimate and reduced to the proposer's decimated input,
    so only the bf16 inputs (2 ld values per pair) and the labels are kept."""
    torch = ctx.torch
    xdec = torch.empty((npairs, 2, model.ld), dtype=torch.int16, device="cuda")
    labels = torch.empty(npairs, dtype=torch.int32, device="cuda")
    at = 0
    for k, (x, y) in enumerate(chunks):
        specs = device_specs(x, y, bits, lag_lo, lag_hi)
        pk = plain_peaks(ctx, specs)
        b = len(specs)
        xdec[at:at + b] = model.prepare(specs)
        labels[at:at + b] = torch.from_numpy(bins_of_lags(pk["lag"], model.nbins)).cuda()
        at += b
        if log and (k % 32 == 0 or at == npairs):
            log(f"[learned] dataset: {at} of {npairs} pairs")
        if at >= npairs:
            break
    return xdec[:at], labels[:at]


def train(ctx, model, xdec, labels, epochs: int, batch: int, lr, seed: int = 0, log=None, loss_every: int = 64):
    """Adam over shuffled mini-batches; lr is a number or one value per
    epoch. Returns the mean loss per epoch (sampled every loss_every steps)."""
    torch = ctx.torch
    n = xdec.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    lrs = list(lr) if isinstance(lr, (list, tuple)) else [lr] * epochs
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        tot, cnt = 0.0, 0
        nsteps = n // batch
        for k, s in enumerate(range(0, n - batch + 1, batch)):
            idx = perm[s:s + batch]
            want = k % loss_every == 0
            loss = model.train_step(xdec[idx].contiguous(), labels[idx].contiguous(), lrs[ep], want_loss=want)
            if want:
                tot += loss
                cnt += 1
            if log and k and k % max(nsteps // 8, 1) == 0:
                log(f"[learned] epoch {ep} step {k}/{nsteps}: loss {tot / max(cnt, 1):.4f}")
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"[learned] epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def proposals(model, xdec, topk: int):
    _, top, margin = model.forward(xdec, topk=topk)
    return top.cpu().numpy(), margin.cpu().numpy()


def window_misses(top, margin, truth_lags, theta: float, nbins: int):
    """Pairs whose windows (margin >= theta) miss the exact lag: counted as
    misses; pairs below theta fall back to the full range and cannot miss."""
    tb = bins_of_lags(truth_lags, nbins)
    use = margin >= theta
    hit = (top == tb[:, None]).any(axis=1)
    return int(np.count_nonzero(use & ~hit)), int(np.count_nonzero(~use))


def tune_threshold(top, margin, truth_lags, nbins: int, max_miss: float = 0.0, min_fallback: float = 0.0):
    """Threshold from a validation set: just above the largest margin of a
    window miss beyond the allowed max_miss share, and at least the
    min_fallback quantile of the margins (a safety share of pairs always
    takes the full range)."""
    tb = bins_of_lags(truth_lags, nbins)
    hit = (top == tb[:, None]).any(axis=1)
    miss_m = np.sort(margin[~hit])[::-1]
    allowed = int(np.floor(max_miss * len(margin)))
    th = float("-inf")
    if miss_m.size > allowed:
        th = float(np.nextafter(np.float32(miss_m[allowed]), np.float32(np.inf)))
    if min_fallback > 0:
        th = max(th, float(np.quantile(margin, min_fallback)))
    return th
