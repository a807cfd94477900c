"""CPU oracle of the learned lag-window proposer (float64, plain numpy).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``): only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` may
use it; it shares no code with the HIP library.

The proposer is not part of the paper; it narrows the lag range on which the
paper's exact integer correlation (Algorithm 1, correlation step) is evaluated. The
network, written out:

* input: each signal of N = 16 Ld samples is reduced to Ld block means of 16
  samples, scaled by 1/sigma of the quantizer (sigma = 6 / ((2K+1) inv_step)),
  so the input has unit power for any gain;
* encoder, shared by both signals: ``layers`` blocks of
  conv1d (kernel 9, zero padding 4, C output channels, bias) -> ReLU ->
  average pooling of 2 -> features F = Ld / 2^layers long;
* head: logits[k] = alpha * sum_c sum_t Fx[c, t] Fy[c, t + k - nbins/2],
  k in [0, nbins) (the correlation of the feature maps, zero outside);
* training: softmax cross-entropy against the bin of the exact lag, Adam.

Gradients are derived by hand (no autograd) and pinned by finite differences
in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

KW = 9          # kernel width
PAD = 4         # zero padding each side


@dataclass(frozen=True)
class Shape:
    ld: int = 16384      # decimated input length
    c: int = 32          # channels
    layers: int = 4
    nbins: int = 512     # head lags (feature steps), centred

    @property
    def f(self) -> int:
        return self.ld >> self.layers

    @property
    def cin(self):
        return [1] + [self.c] * (self.layers - 1)


def param_sizes(s: Shape):
    """(name, shape) of every parameter, in the flat order of the model blob."""
    out = []
    for l, ci in enumerate(s.cin):
        out.append((f"W{l}", (s.c, ci, KW)))
        out.append((f"b{l}", (s.c,)))
    out.append(("alpha", ()))
    return out


def n_params(s: Shape) -> int:
    return sum(int(np.prod(sh)) if sh else 1 for _, sh in param_sizes(s))


def unflatten(s: Shape, flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == n_params(s)
    p, o = {}, 0
    for name, sh in param_sizes(s):
        k = int(np.prod(sh)) if sh else 1
        p[name] = flat[o:o + k].reshape(sh) if sh else float(flat[o])
        o += k
    return p


def flatten(s: Shape, p) -> np.ndarray:
    parts = []
    for name, sh in param_sizes(s):
        parts.append(np.atleast_1d(np.asarray(p[name], dtype=np.float64)).ravel())
    return np.concatenate(parts)


# ------------------------------------------------------------------ input --

def decimate(x, inv_step: float, kmax: int, ld: int):
    """Block means of 16 samples times 1/sigma, sigma = 6 / ((2K+1) inv_step)."""
    x = np.asarray(x, dtype=np.float64)
    assert x.size == 16 * ld
    scale = float(np.float32(inv_step)) * 6.0 / (2 * kmax + 1)
    return x.reshape(ld, 16).mean(axis=1) * scale


def round_params(s: Shape, p, fn):
    """Apply ``fn`` to every weight and bias (not alpha)."""
    return {k: (fn(v) if k != "alpha" else v) for k, v in p.items()}


def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- forward --

def conv_fwd(X, W, b):
    """Z[o, t] = b[o] + sum_i sum_k W[o, i, k] X[i, t + k - 4], zero padded."""
    cin, L = X.shape
    Xp = np.zeros((cin, L + 2 * PAD))
    Xp[:, PAD:PAD + L] = X
    Z = np.tile(np.asarray(b, dtype=np.float64)[:, None], (1, L))
    for k in range(KW):
        Z += W[:, :, k] @ Xp[:, k:k + L]
    return Z


def relu_pool_fwd(Z):
    A = np.maximum(Z, 0.0)
    P = 0.5 * (A[:, 0::2] + A[:, 1::2])
    return A, P


def encoder_fwd(s: Shape, p, xd, store=None):
    """Returns the features and the cache (input and pre-activation per layer).
    ``store`` (e.g. ``bf16_round``) is applied to every stored activation (the
    layer outputs), modelling a device that keeps activations in a narrower
    format; the arithmetic itself stays float64."""
    X = np.asarray(xd, dtype=np.float64)[None, :]
    cache = []
    for l in range(s.layers):
        Z = conv_fwd(X, p[f"W{l}"], p[f"b{l}"])
        A, P = relu_pool_fwd(Z)
        cache.append((X, Z))
        X = store(P) if store is not None else P
    return X, cache


def head_raw(s: Shape, Fx, Fy):
    """raw[k] = sum_c sum_t Fx[c, t] Fy[c, t + k - nbins/2]."""
    F = Fx.shape[1]
    raw = np.zeros(s.nbins)
    h = s.nbins // 2
    for k in range(s.nbins):
        sh = k - h
        lo, hi = max(0, -sh), min(F, F - sh)
        if hi > lo:
            raw[k] = float(np.sum(Fx[:, lo:hi] * Fy[:, lo + sh:hi + sh]))
    return raw


def forward(s: Shape, p, xd, yd, store=None):
    Fx, cx = encoder_fwd(s, p, xd, store)
    Fy, cy = encoder_fwd(s, p, yd, store)
    raw = head_raw(s, Fx, Fy)
    return p["alpha"] * raw, (Fx, Fy, cx, cy, raw)


def softmax_ce(logits, label: int):
    z = logits - logits.max()
    e = np.exp(z)
    prob = e / e.sum()
    loss = -np.log(prob[label])
    g = prob.copy()
    g[label] -= 1.0
    return loss, g


# --------------------------------------------------------------- backward --

def head_bwd(s: Shape, p, Fx, Fy, raw, dlog):
    """Gradients of logits = alpha * raw wrt Fx, Fy and alpha."""
    F = Fx.shape[1]
    h = s.nbins // 2
    a = p["alpha"]
    dFx = np.zeros_like(Fx)
    dFy = np.zeros_like(Fy)
    for k in range(s.nbins):
        sh = k - h
        lo, hi = max(0, -sh), min(F, F - sh)
        if hi > lo:
            dFx[:, lo:hi] += a * dlog[k] * Fy[:, lo + sh:hi + sh]
            dFy[:, lo + sh:hi + sh] += a * dlog[k] * Fx[:, lo:hi]
    dalpha = float(np.dot(dlog, raw))
    return dFx, dFy, dalpha


def conv_bwd(X, W, Z, dP):
    """Through pooling and ReLU, then the convolution: dX, dW, db."""
    cin, L = X.shape
    dA = np.repeat(0.5 * dP, 2, axis=1)
    dZ = dA * (Z > 0)
    Xp = np.zeros((cin, L + 2 * PAD))
    Xp[:, PAD:PAD + L] = X
    dW = np.zeros_like(W)
    for k in range(KW):
        dW[:, :, k] = dZ @ Xp[:, k:k + L].T
    db = dZ.sum(axis=1)
    dXp = np.zeros((cin, L + 2 * PAD))
    for k in range(KW):
        dXp[:, k:k + L] += W[:, :, k].T @ dZ
    return dXp[:, PAD:PAD + L], dW, db


def encoder_bwd(s: Shape, p, cache, dF, grads):
    d = dF
    for l in reversed(range(s.layers)):
        X, Z = cache[l]
        dX, dW, db = conv_bwd(X, p[f"W{l}"], Z, d)
        grads[f"W{l}"] += dW
        grads[f"b{l}"] += db
        d = dX
    return d


def loss_and_grads(s: Shape, p, xd, yd, label: int, store=None):
    logits, (Fx, Fy, cx, cy, raw) = forward(s, p, xd, yd, store)
    loss, dlog = softmax_ce(logits, label)
    grads = {name: np.zeros(sh) if sh else 0.0 for name, sh in param_sizes(s)}
    dFx, dFy, dalpha = head_bwd(s, p, Fx, Fy, raw, dlog)
    grads["alpha"] = dalpha
    encoder_bwd(s, p, cx, dFx, grads)
    encoder_bwd(s, p, cy, dFy, grads)
    return loss, grads, logits


def batch_loss_and_grads(s: Shape, p, xds, yds, labels, store=None):
    """Mean loss and mean gradients over a batch."""
    B = len(labels)
    tot = {name: np.zeros(sh) if sh else 0.0 for name, sh in param_sizes(s)}
    L = 0.0
    logits = []
    for b in range(B):
        loss, g, lg = loss_and_grads(s, p, xds[b], yds[b], int(labels[b]), store)
        L += loss
        logits.append(lg)
        for k in tot:
            tot[k] = tot[k] + g[k]
    return L / B, {k: v / B for k, v in tot.items()}, np.array(logits)


def adam_step(flat, gflat, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), all arrays flat; returns new copies."""
    m = b1 * m + (1 - b1) * gflat
    v = b2 * v + (1 - b2) * gflat * gflat
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------- proposal --

def topk_margin(logits, k: int):
    """Top-k bins (descending logit, ties to the smaller bin) and the margin
    logit_(1) - logit_(k+1)."""
    order = np.lexsort((np.arange(logits.size), -logits))
    top = order[:k]
    margin = float(logits[order[0]] - logits[order[k]]) if logits.size > k else float("inf")
    return top, margin


def label_of_lag(lag: int, nbins: int, width: int) -> int:
    """Bin of a lag: floor((lag + nbins/2 * width) / width), clamped."""
    return int(np.clip((lag + (nbins // 2) * width) // width, 0, nbins - 1))


def windowed_argmax(u, v, bins, width: int, nbins: int):
    """Argmax (smallest lag, max, count) of Eq. (1) over the union of the given
    bins, each the lags [(b - nbins/2) width, (b - nbins/2 + 1) width); the
    bins are distinct, so their union is their disjoint sum."""
    from . import xcorr_at
    lags = np.concatenate([np.arange((b - nbins // 2) * width, (b - nbins // 2 + 1) * width) for b in sorted(bins)])
    r = xcorr_at(u, v, lags)
    best = r.max()
    sel = lags[r == best]
    return int(sel.min()), int(best), int(sel.size)
