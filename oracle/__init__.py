"""CPU oracle for the exact integer time-difference estimator.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the HIP library (``paper_2509_19974_amd``) and never imports it.

What it computes is the plain definition of each step, written out:

* ``sumsq`` / ``inv_step`` -- the per-signal scale of the uniform quantizer
  (the paper leaves the quantizer free, Section 3.2; the library fixes a
  symmetric mid-tread quantizer on [-3 sigma, 3 sigma]). S = sum of x^2 is
  the exact real sum rounded once to float64 (``math.fsum`` of the squares,
  each exact in float64), so it depends on no summation order.
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
  tie-refinement step. The refinement compares the exact real values of
  Eq. (1) at the tied lags: every product x[m] y[m + tau] of float32 samples
  is exact in float64, and the sign of the exactly rounded sum of the
  products at one lag minus those at another (``math.fsum``) is the sign of
  the exact difference.
* ``stream`` -- correlation of a stream against a template, block by block
  (the streaming extension named as future work in Section 5): the plain
  correlation of Eq. (1) over the concatenated stream, cut into the lags each
  push makes final, with per-block and running argmaxes.
* ``xcorr_long_certified`` -- for signals too long for the direct sum over all
  lags: a float64 radix-2 FFT correlation of the integer sequences (plain C,
  ``oracle_conv_fft``), rounded to the nearest integer and accepted only when
  Percival's a-priori bound on the FFT-product error is below one half (so
  the rounding is provably exact), and cross-checked by direct sums on a lag
  subset.

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
    lib.oracle_conv_fft.argtypes = [vp, i64, vp, i64, i64, vp, vp]
    lib.oracle_conv_fft.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads used by the direct sums."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Threads for later direct sums (timing only; results do not depend on it)."""
    _load().oracle_set_threads(int(n))


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


def sumsq(x) -> float:
    """S = sum of x[m]^2 over the finite samples, as the exact real sum
    rounded once to float64 (round to nearest, ties to even). Each square of
    a float32 is exact in float64; ``math.fsum`` returns the correctly
    rounded sum of its float64 inputs, so S depends on no summation order."""
    x = _f32(x).astype(np.float64)
    x = x[np.isfinite(x)]
    return math.fsum((x * x).tolist())


def inv_step_from_sumsq(S: float, n: int, bits: int) -> float:
    """fl32((2K+1) / (6 sigma)), sigma = sqrt(S/n) (float64 operations, each
    correctly rounded); 0.0 when S == 0."""
    return float(np.float32(_load().oracle_inv_step_from_sumsq(float(S), int(n), bits)))


def inv_step(x, bits: int) -> float:
    """The uniform quantizer's automatic scale of a signal (see ``sumsq``)."""
    x = _f32(x)
    return inv_step_from_sumsq(sumsq(x), x.size, bits)


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


def _products(x64, y64, tau: int) -> np.ndarray:
    """x[m] y[m + tau] over the overlap, ascending m (each exact in float64)."""
    lo = max(0, -tau)
    hi = min(x64.size, y64.size - tau)
    if hi <= lo:
        return np.zeros(0)
    return x64[lo:hi] * y64[lo + tau:hi + tau]


def compare_real_xcorr(x, y, tau_a: int, tau_b: int) -> int:
    """Sign (-1, 0, +1) of (x * y)[tau_a] - (x * y)[tau_b], Eq. (1) on the
    float signals, decided exactly: the products are exact in float64, and
    ``math.fsum`` of the products at tau_a and the negated products at tau_b
    is the exact difference rounded once, whose sign is exact (a non-zero
    difference of multiples of 2^-298 rounds to a non-zero float64). The
    overlaps must hold finite samples only."""
    return _compare64(_f32(x).astype(np.float64), _f32(y).astype(np.float64), tau_a, tau_b)


def _compare64(x64, y64, tau_a: int, tau_b: int) -> int:
    d = math.fsum(_products(x64, y64, tau_a).tolist() + (-_products(x64, y64, tau_b)).tolist())
    return (d > 0) - (d < 0)


def real_xcorr_finite(x, y, tau: int) -> bool:
    """True when every sample of x and y in the overlap at tau is finite."""
    x, y = _f32(x), _f32(y)
    lo = max(0, -tau)
    hi = min(x.size, y.size - tau)
    if hi <= lo:
        return True
    return bool(np.all(np.isfinite(x[lo:hi])) and np.all(np.isfinite(y[lo + tau:hi + tau])))


def refine_ties(x, y, tied):
    """Algorithm 1, tie-refinement step: among the tied lags (ascending), the
    set whose exact real correlation (Eq. (1) on x, y) is largest, in
    ascending order. Reading for non-finite samples (not in the paper): if
    any tied lag's overlap holds a NaN or Inf sample, its real correlation is
    not a real number and the lags cannot be compared; the tied set is then
    returned unchanged. Returns (refined set, compared) with compared False
    in that case."""
    tied = [int(t) for t in tied]
    if len(tied) <= 1:
        return tied, True
    if not all(real_xcorr_finite(x, y, t) for t in tied):
        return tied, False
    x64 = _f32(x).astype(np.float64)
    y64 = _f32(y).astype(np.float64)
    best = [tied[0]]
    for t in tied[1:]:
        c = _compare64(x64, y64, t, best[0])
        if c > 0:
            best = [t]
        elif c == 0:
            best.append(t)
    return best, True


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
                     inv_step_x: float | None = None, inv_step_y: float | None = None,
                     max_ties: int | None = None):
    """Algorithm 1 with its tie-refinement step: ties of the integer
    correlation are resolved by the exact real correlation of the unquantized
    signals at the tied lags (``refine_ties``). With max_ties, only the
    smallest max_ties tied lags take part (the library's partial refinement).
    Returns the argmax-step result plus ``lag_set`` (sorted), ``refined``
    (False when non-finite samples prevented the comparison) and ``partial``."""
    res = estimate(x, y, bits, lag_lo, lag_hi, inv_step_x, inv_step_y)
    r = res["r"]
    tied = (np.nonzero(r == res["rmax"])[0].astype(np.int64) + lag_lo).tolist()
    res["partial"] = max_ties is not None and len(tied) > max_ties
    if res["partial"]:
        tied = tied[:max_ties]
    res["lag_set"], res["refined"] = refine_ties(x, y, tied)
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
    """A-priori bound on the max-norm error of the float64 FFT product in
    ``oracle_conv_fft`` (radix-2 complex transforms of length N = 2^k, three
    transforms and one pointwise product): Percival's bound for FFT-based
    multiplication (C. Percival, Math. Comp. 72 (2003); restated by Brent and
    Zimmermann, Modern Computer Arithmetic, Section 3.3),
        ||z' - z||_inf < ||u||_2 ||v||_2 ((1+e)^(3k) (1+e sqrt5)^(3k+1) (1+b)^(3k) - 1),
    with e = 2^-53 the unit roundoff, sqrt(5) e the error of a complex
    product computed with four real products, and b the twiddle error (2 e:
    the twiddles are long-double values rounded once). The norms are exact
    integers; the bound is evaluated in float64 and inflated by 1% to cover
    its own rounding."""
    nu2 = math.sqrt(float(int(np.dot(u.astype(np.int64), u.astype(np.int64)))))
    nv2 = math.sqrt(float(int(np.dot(v.astype(np.int64), v.astype(np.int64)))))
    k = int(round(math.log2(n_fft)))
    if (1 << k) != n_fft:
        raise ValueError("n_fft must be a power of two")
    e = 2.0 ** -53
    b = 2.0 * e
    growth = math.expm1(3 * k * math.log1p(e) + (3 * k + 1) * math.log1p(e * math.sqrt(5.0))
                        + 3 * k * math.log1p(b))
    return 1.01 * nu2 * nv2 * growth


def conv_fft_f64(u, v, n_fft: int) -> np.ndarray:
    """rev(u) conv v (length nu + nv - 1) through the float64 radix-2 FFT,
    unrounded; entry j approximates r[j - (nu - 1)]."""
    u, v = _i8(u), _i8(v)
    out = np.empty(u.size + v.size - 1, dtype=np.float64)
    scratch = np.empty(5 * n_fft, dtype=np.float64)
    _load().oracle_conv_fft(_ptr(u), u.size, _ptr(v), v.size, n_fft, _ptr(out), _ptr(scratch))
    return out


def xcorr_long_certified(u, v, lag_lo: int, lag_hi: int, check_lags=None):
    """Exact int64 r over [lag_lo, lag_hi] for long sequences.

    The float64 FFT correlation of the integer sequences is rounded to the
    nearest integer; the result is exact when Percival's error bound
    (``fft_rounding_bound``) is below 1/2, which is asserted. The lags in ``check_lags`` are additionally
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
    full = conv_fft_f64(u, v, n)
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
