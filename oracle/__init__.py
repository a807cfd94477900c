"""CPU oracle for the exact integer time-difference estimator.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the HIP library (``paper_2509_19974_amd``) and never imports it.

What it computes is the plain definition of each step, written out:

* ``sumsq_pairwise`` / ``inv_step`` -- the per-signal scale of the uniform
  quantizer (the paper leaves the quantizer free, Section 3.2; the library fixes
  a symmetric mid-tread quantizer on [-3 sigma, 3 sigma] and a pairwise
  float64 sum of squares over a fixed binary tree so that two implementations
  agree bit for bit).
* ``quantize`` -- Algorithm 1, quantization step: monotone integer maps with phi(0) = 0;
  sign with sign(0) = 0 (Section 4.2) for bits = 1.
* ``quantize_nonuniform``, ``mulaw_thresholds``, ``lloyd_max_gauss`` --
  non-uniform maps for b in {2, 4} (Section 3.2 allows any quantizer with
  integer range; Section 5 names better quantizers as future work): the
  cell boundaries of mu-law companding and of the Lloyd-Max quantizer of a
  unit Gaussian, the code being the cell index.
* ``xcorr`` / ``xcorr_at`` -- Algorithm 1, correlation step: Eq. (1) on the integer
  sequences, int64 direct sums.
* ``argmax`` -- Algorithm 1, argmax step: maximum, smallest maximising lag and the
  number of maximisers (Remark 1).
* ``xcorr_f64_at`` -- Eq. (1) on the unquantized signals in float64.
* ``estimate`` / ``estimate_refined`` -- Algorithm 1 without, and with, its
  tie-refinement step.
* ``stream`` -- correlation of a stream against a template, block by block
  (the streaming extension named as future work in Section 5): the plain
  correlation of Eq. (1) over the concatenated stream, cut into the lags each
  push makes final, with per-block and running argmaxes.
* ``xcorr_long_certified`` -- for signals too long for the direct sum over all
  lags: a float64 FFT correlation of the integer sequences, rounded to the
  nearest integer, accepted only under an a-priori rounding-error bound below
  one half (so the rounding is provably exact), and cross-checked by direct
  sums on a lag subset.

Everything heavy runs in ``tde_oracle.c`` (plain loops, int64/float64),
compiled with gcc and loaded through ctypes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tde_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libtde_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, OpenMP for the lag loop)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, f32, f64, vp = ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p
    lib.oracle_sumsq_pairwise.argtypes = [vp, i64, vp]
    lib.oracle_sumsq_pairwise.restype = f64
    lib.oracle_kmax.argtypes = [ctypes.c_int]
    lib.oracle_kmax.restype = ctypes.c_int
    lib.oracle_inv_step_from_sumsq.argtypes = [f64, i64, ctypes.c_int]
    lib.oracle_inv_step_from_sumsq.restype = f32
    lib.oracle_quantize.argtypes = [vp, i64, ctypes.c_int, f32, vp]
    lib.oracle_quantize.restype = i64
    lib.oracle_xcorr_i64.argtypes = [vp, i64, vp, i64, i64, i64, vp]
    lib.oracle_xcorr_i64.restype = None
    lib.oracle_xcorr_i64_at.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    lib.oracle_xcorr_i64_at.restype = None
    lib.oracle_argmax_i64.argtypes = [vp, i64, i64, vp, vp, vp]
    lib.oracle_argmax_i64.restype = None
    lib.oracle_xcorr_f64_at.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    lib.oracle_xcorr_f64_at.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads used by the direct sums."""
    return int(_load().oracle_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32)


def _i8(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.int8)


# ---------------------------------------------------------------- scale ----

def kmax(bits: int) -> int:
    """Largest code magnitude: 1 for sign (ternary), 2^(b-1)-1 otherwise."""
    if bits not in (1, 2, 4, 8):
        raise ValueError("bits must be 1, 2, 4 or 8")
    return int(_load().oracle_kmax(bits))


def sumsq_pairwise(x) -> float:
    """Pairwise (fixed binary tree) float64 sum of the exact squares of the
    finite samples, zero-padded to a power-of-two length."""
    x = _f32(x)
    n = x.size
    p2 = 1
    while p2 < n:
        p2 *= 2
    scratch = np.zeros(p2, dtype=np.float64)
    return float(_load().oracle_sumsq_pairwise(_ptr(x), n, _ptr(scratch)))


def inv_step(x, bits: int) -> float:
    """fl32((2K+1) / (6 sigma)), sigma = sqrt(S/n); 0.0 when S == 0."""
    x = _f32(x)
    S = sumsq_pairwise(x)
    return float(np.float32(_load().oracle_inv_step_from_sumsq(S, x.size, bits)))


# ------------------------------------------------------------- quantize ----

def quantize(x, bits: int, inv_step_value: float | None = None):
    """Algorithm 1, quantization step. Returns (q int8, n_nonfinite, inv_step used)."""
    x = _f32(x)
    if bits not in (1, 2, 4, 8):
        raise ValueError("bits must be 1, 2, 4 or 8")
    if bits == 1:
        s = 0.0
    elif inv_step_value is None or inv_step_value <= 0:
        s = inv_step(x, bits)
    else:
        s = float(np.float32(inv_step_value))
    q = np.empty(x.size, dtype=np.int8)
    nf = _load().oracle_quantize(_ptr(x), x.size, bits, s, _ptr(q))
    return q, int(nf), s


# ------------------------------------------------ non-uniform quantizers ----
# Quantizer kinds: 0 uniform (above), 1 mu-law (mu = 255), 2 Lloyd-Max for a
# unit Gaussian. Every kind uses the uniform quantizer's scale
# inv_step = fl32((2K+1)/(6 sigma)) and the scaled sample z = fl32(x inv_step)
# (z = +-(K + 1/2) at +-3 sigma); the code is sign(z) times the number of cell
# boundaries T_1 < ... < T_K (in units of z) strictly below |z|. NaN gives 0,
# +-Inf gives +-K, inv_step = 0 gives 0. Monotone with phi(0) = 0 (Theorem 1).

MU = 255.0


def mulaw_thresholds(K: int, mu: float = MU) -> np.ndarray:
    """Cell boundaries (units of sigma) of mu-law companding on [-3 sigma,
    3 sigma]: the compressor c(a) = ln(1 + mu a / 3) / ln(1 + mu) maps a
    magnitude a (in sigma) to [0, 1], cut uniformly into K + 1/2 cells, so the
    k-th boundary solves c(a) = (k - 1/2) / (K + 1/2)."""
    return np.array([3.0 * ((1.0 + mu) ** ((k - 0.5) / (K + 0.5)) - 1.0) / mu for k in range(1, K + 1)])


def _phi(t: float) -> float:
    return math.exp(-0.5 * t * t) / math.sqrt(2.0 * math.pi)


def _Phi(t: float) -> float:
    return 0.5 * math.erfc(-t / math.sqrt(2.0))


def lloyd_max_gauss(K: int, tol: float = 1e-15, max_iter: int = 100000):
    """Lloyd-Max quantizer of a unit Gaussian with 2K+1 levels (0 and +-y_k):
    each boundary t_k is the midpoint of its two levels, each level the
    centroid E[X | t_k <= X < t_(k+1)] = (phi(t_k) - phi(t_(k+1))) /
    (Phi(t_(k+1)) - Phi(t_k)) with t_(K+1) = inf. Lloyd's iteration from the
    uniform levels k 6/(2K+1), until no level moves by more than tol.
    Returns (boundaries t_1..t_K, levels y_1..y_K), in units of sigma."""
    y = [0.0] + [k * 6.0 / (2 * K + 1) for k in range(1, K + 1)]
    for _ in range(max_iter):
        t = [0.0] + [(y[k - 1] + y[k]) / 2.0 for k in range(1, K + 1)]
        ny = [0.0]
        for k in range(1, K + 1):
            a = t[k]
            if k < K:
                b = t[k + 1]
                ny.append((_phi(a) - _phi(b)) / (_Phi(b) - _Phi(a)))
            else:
                ny.append(_phi(a) / (1.0 - _Phi(a)))
        moved = max(abs(p - q) for p, q in zip(y, ny))
        y = ny
        if moved <= tol:
            break
    t = [(y[k - 1] + y[k]) / 2.0 for k in range(1, K + 1)]
    return np.array(t), np.array(y[1:])


def nonuniform_table(kind: int, bits: int) -> np.ndarray:
    """float32 cell boundaries T_k in units of z = x inv_step (sigma units
    times (2K+1)/6) for kind 1 (mu-law) or 2 (Lloyd-Max Gaussian), bits 2 or 4."""
    if bits not in (2, 4):
        raise ValueError("non-uniform quantizers are defined for bits 2 and 4")
    K = kmax(bits)
    t = mulaw_thresholds(K) if kind == 1 else lloyd_max_gauss(K)[0]
    return np.array([np.float32(v * (2 * K + 1) / 6.0) for v in t], dtype=np.float32)


def quantize_nonuniform(x, bits: int, kind: int, inv_step_value: float | None = None):
    """Algorithm 1, quantization step with a non-uniform monotone map (kind 1 or 2; bits
    1 is sign for every kind). Returns (q int8, n_nonfinite, inv_step used)."""
    x = _f32(x)
    if bits == 1 or kind == 0:
        return quantize(x, bits, inv_step_value)
    T = nonuniform_table(kind, bits)
    if inv_step_value is None or inv_step_value <= 0:
        s = inv_step(x, bits)
    else:
        s = float(np.float32(inv_step_value))
    nonfinite = int(np.count_nonzero(~np.isfinite(x)))
    q = np.zeros(x.size, dtype=np.int8)
    if s == 0.0:
        return q, nonfinite, s
    with np.errstate(invalid="ignore", over="ignore"):
        z = x * np.float32(s)                       # float32 product, rounded to nearest even
    ok = ~np.isnan(z)
    a = np.abs(z[ok])
    code = np.zeros(a.size, dtype=np.int64)
    for t in T:
        code += (a > t).astype(np.int64)
    q[ok] = (np.sign(z[ok]).astype(np.int64) * code).astype(np.int8)
    return q, nonfinite, s


# ---------------------------------------------------------- correlation ----

def xcorr(u, v, lag_lo: int, lag_hi: int) -> np.ndarray:
    """Eq. (1) on integer sequences: r[i] = sum_m u[m] v[m + lag_lo + i], int64."""
    u, v = _i8(u), _i8(v)
    if lag_hi < lag_lo:
        raise ValueError("lag_hi < lag_lo")
    r = np.empty(lag_hi - lag_lo + 1, dtype=np.int64)
    _load().oracle_xcorr_i64(_ptr(u), u.size, _ptr(v), v.size, lag_lo, lag_hi, _ptr(r))
    return r


def xcorr_at(u, v, lags) -> np.ndarray:
    """Eq. (1) at a list of lags, int64 direct sums."""
    u, v = _i8(u), _i8(v)
    lags = np.ascontiguousarray(lags, dtype=np.int64)
    r = np.empty(lags.size, dtype=np.int64)
    _load().oracle_xcorr_i64_at(_ptr(u), u.size, _ptr(v), v.size, _ptr(lags), lags.size, _ptr(r))
    return r


def argmax(r, lag_lo: int):
    """Algorithm 1, argmax step: (smallest maximising lag, max value, #maximisers)."""
    r = np.ascontiguousarray(r, dtype=np.int64)
    if r.size == 0:
        raise ValueError("empty lag range")
    lag, rmax, nt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _load().oracle_argmax_i64(_ptr(r), r.size, lag_lo, ctypes.byref(lag),
                              ctypes.byref(rmax), ctypes.byref(nt))
    return int(lag.value), int(rmax.value), int(nt.value)


def xcorr_f64_at(x, y, lags) -> np.ndarray:
    """Eq. (1) on the float signals in float64, ascending-m summation."""
    x, y = _f32(x), _f32(y)
    lags = np.ascontiguousarray(lags, dtype=np.int64)
    r = np.empty(lags.size, dtype=np.float64)
    _load().oracle_xcorr_f64_at(_ptr(x), x.size, _ptr(y), y.size, _ptr(lags), lags.size, _ptr(r))
    return r


def xcorr_f64_at_pairwise(x, y, lags) -> np.ndarray:
    """Eq. (1) on the float signals in float64 with a fixed summation order:
    the products x[m] y[m + tau] (exact in float64) over the overlap, in
    ascending m, zero-padded to a power-of-two length and added as a binary
    tree (adjacent pairs, level by level). Used for the tie refinement of
    Algorithm 1, tie-refinement step, so that the choice between tied lags is made in
    the same arithmetic on every implementation."""
    x = np.asarray(_f32(x), dtype=np.float64)
    y = np.asarray(_f32(y), dtype=np.float64)
    out = []
    for tau in np.asarray(lags, dtype=np.int64).tolist():
        lo = max(0, -tau)
        hi = min(x.size, y.size - tau)
        if hi <= lo:
            out.append(0.0)
            continue
        p = x[lo:hi] * y[lo + tau:hi + tau]
        n = 1
        while n < p.size:
            n *= 2
        a = np.zeros(n)
        a[:p.size] = p
        while a.size > 1:
            a = a[0::2] + a[1::2]
        out.append(float(a[0]))
    return np.array(out)


def overlap_count(nu: int, nv: int, tau: int) -> int:
    """#{m : 0 <= m < nu, 0 <= m + tau < nv}."""
    return max(0, min(nu, nv - tau) - max(0, -tau))


# ------------------------------------------------------------- Alg. 1 -----

def estimate(x, y, bits: int, lag_lo: int, lag_hi: int,
             inv_step_x: float | None = None, inv_step_y: float | None = None):
    """Algorithm 1 up to its argmax step. Returns a dict with lag, rmax, n_ties, r, q's."""
    u, nfx, sx = quantize(x, bits, inv_step_x)
    v, nfy, sy = quantize(y, bits, inv_step_y)
    r = xcorr(u, v, lag_lo, lag_hi)
    lag, rmax, nt = argmax(r, lag_lo)
    return {"lag": lag, "rmax": rmax, "n_ties": nt, "r": r, "u": u, "v": v,
            "inv_step_x": sx, "inv_step_y": sy, "nonfinite_x": nfx, "nonfinite_y": nfy}


def estimate_refined(x, y, bits: int, lag_lo: int, lag_hi: int,
                     inv_step_x: float | None = None, inv_step_y: float | None = None):
    """Algorithm 1 with its tie-refinement step: ties of the integer correlation are resolved by
    the float64 correlation of the unquantized signals (fixed pairwise
    summation order), evaluated only at the tied lags. Returns the refined
    argmax set (sorted) and the line-4 result."""
    res = estimate(x, y, bits, lag_lo, lag_hi, inv_step_x, inv_step_y)
    r = res["r"]
    tied = np.nonzero(r == res["rmax"])[0].astype(np.int64) + lag_lo
    if tied.size > 1:
        rf = xcorr_f64_at_pairwise(x, y, tied)
        best = rf.max()
        tied = tied[rf == best]
    res["lag_set"] = [int(t) for t in tied]
    return res


# ------------------------------------------------------------ streaming ---

def stream(x, blocks, bits: int, inv_step_y: float, inv_step_x: float | None = None):
    """Correlation of a stream against a template x (nx samples), the stream
    arriving as the float blocks in ``blocks`` (the streaming extension the
    paper names as future work, Section 5).

    The template is quantized once (its own scale, or inv_step_x); the stream
    with one fixed scale inv_step_y for every block, so the quantized stream
    is the quantization of the concatenation (Algorithm 1, quantization step, one
    monotone map). Lags follow Eq. (1) with u = template codes and v = stream
    codes: r[tau] = sum_m u[m] v[m + tau], v zero outside the stream. After a
    push that brings the stream to T samples, the lags tau <= T - nx are
    final (they read v only on [tau, tau + nx), inside [0, T)); a push of B
    samples makes B new lags final, and the finishing step the last nx - 1
    lags [T - nx + 1, T - 1] (zero beyond the end). Returns one record per
    push and one for the finish: the lags, their r, the argmax of those lags
    and the running argmax over every final lag so far (Algorithm 1, argmax step,
    smallest lag on ties)."""
    x = _f32(x)
    nx = x.size
    ys = [_f32(b) for b in blocks]
    if not ys or min(b.size for b in ys) < 1:
        raise ValueError("every block needs at least one sample")
    u, _, sx = quantize(x, bits, inv_step_x)
    v, _, _ = quantize(np.concatenate(ys), bits, inv_step_y)
    T = v.size
    lo_all = -(nx - 1)
    r_all = xcorr(u, v, lo_all, T - 1)            # every lag of the finished stream
    spans, t = [], 0
    for b in ys:
        spans.append((t - nx + 1, t + b.size - nx))
        t += b.size
    spans.append((T - nx + 1, T - 1))
    records = []
    for a, b in spans:
        rec = {"lag_lo": a, "lag_hi": b, "r": r_all[a - lo_all:b - lo_all + 1]}
        rec["block"] = argmax(rec["r"], a) if b >= a else None
        rec["running"] = argmax(r_all[:b - lo_all + 1], lo_all)
        records.append(rec)
    return {"u": u, "v": v, "inv_step_x": sx, "records": records, "r_all": r_all}


# ------------------------------------------------- long-signal route ------

def fft_rounding_bound(u, v, n_fft: int) -> float:
    """A-priori bound on the max-norm error of a float64 FFT convolution of the
    integer sequences u and v with transform length n_fft:
    ||err||_inf <= ||u||_2 ||v||_2 * 3 log2(n) * 8 eps (a generous multiple of
    the standard forward-error estimate for radix-2 FFT convolution)."""
    nu2 = math.sqrt(float(np.dot(u.astype(np.float64), u.astype(np.float64))))
    nv2 = math.sqrt(float(np.dot(v.astype(np.float64), v.astype(np.float64))))
    eps = np.finfo(np.float64).eps
    return nu2 * nv2 * 3.0 * math.log2(n_fft) * 8.0 * eps


def xcorr_long_certified(u, v, lag_lo: int, lag_hi: int, check_lags=None):
    """Exact int64 r over [lag_lo, lag_hi] for long sequences.

    The float64 FFT correlation of the integer sequences is rounded to the
    nearest integer; the result is exact when the rounding-error bound is
    below 1/2, which is asserted. The lags in ``check_lags`` are additionally
    recomputed by direct int64 sums and must agree."""
    u, v = _i8(u), _i8(v)
    nu, nv = u.size, v.size
    n = 1
    while n < nu + nv - 1:
        n *= 2
    bound = fft_rounding_bound(u, v, n)
    if not bound < 0.5:
        raise ArithmeticError(f"FFT rounding bound {bound} not below 1/2")
    # r[tau] = sum_m u[m] v[m+tau]; with ur = reversed u, (ur conv v)[j] = r[j - (nu-1)]
    ur = u[::-1].astype(np.float64)
    full = np.fft.irfft(np.fft.rfft(ur, n) * np.fft.rfft(v.astype(np.float64), n), n)
    full = full[: nu + nv - 1]
    rounded = np.rint(full)
    taus = np.arange(lag_lo, lag_hi + 1, dtype=np.int64)
    idx = taus + (nu - 1)
    r = np.zeros(taus.size, dtype=np.int64)
    ok = (idx >= 0) & (idx < nu + nv - 1)
    r[ok] = rounded[idx[ok]].astype(np.int64)
    if check_lags is not None:
        check_lags = np.ascontiguousarray(check_lags, dtype=np.int64)
        direct = xcorr_at(u, v, check_lags)
        got = r[check_lags - lag_lo]
        if not np.array_equal(direct, got):
            raise ArithmeticError("certified FFT route disagrees with direct sums")
    return r
