"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a library
routine that computes the same quantity, the paper's own Kronecker-substitution
route (Section 3.2), closed-form identities, the invariance theorem
(Theorem 1) on exact shifts, or hand-derived tiny cases.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth


def rand_q(rng, n, k, p_zero=0.1):
    return synth.random_int_seq(rng, n, k, p_zero)


# ------------------------------------------------------------ correlation --

@pytest.mark.parametrize("nu,nv", [(1, 1), (1, 7), (7, 1), (5, 9), (33, 17), (300, 301), (1000, 64)])
@pytest.mark.parametrize("k", [1, 7, 127])
def test_xcorr_full_equals_numpy_correlate(nu, nv, k):
    """numpy.correlate(v, u, 'full')[j] = sum_n v[n + j - (nu-1)] u[n] (exact int64)."""
    rng = np.random.default_rng(nu * 1000 + nv + k)
    u, v = rand_q(rng, nu, k), rand_q(rng, nv, k)
    r = oracle.xcorr(u, v, -(nu - 1), nv - 1)
    ref = np.correlate(v.astype(np.int64), u.astype(np.int64), "full")
    assert r.dtype == np.int64
    np.testing.assert_array_equal(r, ref)


def test_xcorr_is_convolution_with_reversal():
    """Section 3.2: correlation = convolution with one signal reversed."""
    rng = np.random.default_rng(3)
    u, v = rand_q(rng, 211, 127), rand_q(rng, 97, 127)
    r = oracle.xcorr(u, v, -(u.size - 1), v.size - 1)
    conv = np.convolve(u[::-1].astype(np.int64), v.astype(np.int64))
    np.testing.assert_array_equal(r, conv)


def _kronecker_product(a, b, k):
    """Section 3.2: evaluate both polynomials at 2^L with 2^L > 2 N K^2, one
    big-integer product, then read off the signed coefficients."""
    n = max(len(a), len(b))
    L = int(math.floor(math.log2(n * k * k))) + 2
    assert 2 ** L > 2 * n * k * k
    A = sum(int(c) << (L * i) for i, c in enumerate(a))
    B = sum(int(c) << (L * i) for i, c in enumerate(b))
    W = A * B
    out = []
    half, full = 1 << (L - 1), 1 << L
    for _ in range(len(a) + len(b) - 1):
        c = W & (full - 1)
        if c >= half:
            c -= full
        out.append(c)
        W = (W - c) >> L
    assert W == 0
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("n,k", [(8, 1), (64, 7), (500, 127), (4096, 1), (2048, 7)])
def test_xcorr_equals_kronecker_substitution(n, k):
    rng = np.random.default_rng(n + k)
    u, v = rand_q(rng, n, k), rand_q(rng, n + 3, k)
    r = oracle.xcorr(u, v, -(u.size - 1), v.size - 1)
    ks = _kronecker_product(u[::-1], v, k)
    np.testing.assert_array_equal(r, ks)


@pytest.mark.parametrize("nu,nv,k", [(1, 1, 1), (17, 40, 7), (1000, 999, 127), (4099, 4096, 127)])
def test_xcorr_sum_and_moment_identities(nu, nv, k):
    """sum_tau r = (sum u)(sum v); sum_tau tau r = (sum u)(sum k v_k) - (sum m u_m)(sum v)."""
    rng = np.random.default_rng(nu + 7 * nv)
    u, v = rand_q(rng, nu, k), rand_q(rng, nv, k)
    r = oracle.xcorr(u, v, -(nu - 1), nv - 1)
    taus = np.arange(-(nu - 1), nv, dtype=object)
    su, sv = int(u.astype(np.int64).sum()), int(v.astype(np.int64).sum())
    mu = int((np.arange(nu) * u.astype(np.int64)).sum())
    mv = int((np.arange(nv) * v.astype(np.int64)).sum())
    assert int(r.sum()) == su * sv
    assert int((taus * r.astype(object)).sum()) == su * mv - mu * sv


def test_xcorr_partial_lag_range_and_outside_support():
    rng = np.random.default_rng(11)
    u, v = rand_q(rng, 50, 7), rand_q(rng, 70, 7)
    full = oracle.xcorr(u, v, -200, 200)
    # outside the support the correlation is zero
    taus = np.arange(-200, 201)
    outside = (taus < -(u.size - 1)) | (taus > v.size - 1)
    assert np.all(full[outside] == 0)
    sub = oracle.xcorr(u, v, -13, 29)
    np.testing.assert_array_equal(sub, full[200 - 13:200 + 30])
    at = oracle.xcorr_at(u, v, [-200, -49, 0, 69, 5])
    np.testing.assert_array_equal(at, full[np.array([-200, -49, 0, 69, 5]) + 200])


def test_xcorr_symmetry_bound_and_parity():
    rng = np.random.default_rng(12)
    for k in (1, 7, 127):
        u, v = rand_q(rng, 123, k, 0.3), rand_q(rng, 77, k, 0.3)
        r_uv = oracle.xcorr(u, v, -130, 130)
        r_vu = oracle.xcorr(v, u, -130, 130)
        np.testing.assert_array_equal(r_uv, r_vu[::-1])
        for i, tau in enumerate(range(-130, 131)):
            assert abs(int(r_uv[i])) <= oracle.overlap_count(u.size, v.size, tau) * k * k
    # ternary: every non-zero product is +-1, so r has the parity of their count
    u, v = rand_q(rng, 200, 1, 0.4), rand_q(rng, 180, 1, 0.4)
    r = oracle.xcorr(u, v, -199, 179)
    nzu, nzv = (u != 0).astype(np.int64), (v != 0).astype(np.int64)
    cnt = np.correlate(nzv, nzu, "full")
    assert np.all((r - cnt) % 2 == 0)


def test_xcorr_tiny_hand_derived():
    # u = [1, -1, 1], v = [1, 1]; lags -2..1:
    #  tau=-2: u2 v0 = 1; tau=-1: u1 v0 + u2 v1 = -1 + 1 = 0;
    #  tau= 0: u0 v0 + u1 v1 = 1 - 1 = 0; tau=1: u0 v1 = 1.
    r = oracle.xcorr([1, -1, 1], [1, 1], -2, 1)
    assert r.tolist() == [1, 0, 0, 1]
    assert oracle.argmax(r, -2) == (-2, 1, 2)
    # all-positive x of length 5 delayed by 2 with zero fill, sign-quantized:
    # u = [1,1,1,1,1], v = [0,0,1,1,1]; for 0 <= tau <= 2 the overlap with v's
    # support is 3, so r plateaus at 3 there (a tie, Remark 1); r[-2] = v0 = 0 ... etc.
    r = oracle.xcorr([1] * 5, [0, 0, 1, 1, 1], -4, 4)
    assert r.tolist() == [0, 0, 1, 2, 3, 3, 3, 2, 1]
    assert oracle.argmax(r, -4) == (0, 3, 3)


def test_xcorr_exhaustive_ternary_n3():
    """All 3^3 x 3^3 ternary pairs of length 3 against numpy.correlate."""
    vals = np.array(np.meshgrid(*[[-1, 0, 1]] * 3, indexing="ij")).reshape(3, -1).T
    for u in vals:
        for v in vals[::3]:
            r = oracle.xcorr(u, v, -2, 2)
            np.testing.assert_array_equal(r, np.correlate(v, u, "full"))


# ----------------------------------------------------------------- argmax --

@pytest.mark.parametrize("seed", range(5))
def test_argmax_matches_numpy(seed):
    rng = np.random.default_rng(seed)
    r = rng.integers(-5, 6, size=1000).astype(np.int64)
    lag, rmax, nt = oracle.argmax(r, -500)
    assert rmax == r.max()
    assert lag == -500 + int(np.argmax(r))          # numpy: first occurrence
    assert nt == int(np.count_nonzero(r == r.max()))


def test_argmax_single_and_constant():
    assert oracle.argmax(np.array([7]), 3) == (3, 7, 1)
    assert oracle.argmax(np.zeros(11, dtype=np.int64), -5) == (-5, 0, 11)
    big = np.array([-(2 ** 40), 2 ** 40, 2 ** 40 - 1, 2 ** 40], dtype=np.int64)
    assert oracle.argmax(big, 0) == (1, 2 ** 40, 2)


# -------------------------------------------------------------- quantizer --

@pytest.mark.parametrize("bits", [2, 4, 8])
def test_quantize_uniform_equals_numpy_rint(bits):
    rng = np.random.default_rng(bits)
    x = (rng.standard_normal(20000) * 3).astype(np.float32)
    s = np.float32(1.37)
    q, nf, used = oracle.quantize(x, bits, float(s))
    K = oracle.kmax(bits)
    ref = np.clip(np.rint(x * s), -K, K).astype(np.int8)   # float32 * float32 -> float32
    np.testing.assert_array_equal(q, ref)
    assert nf == 0 and used == float(s)


def test_quantize_sign_equals_numpy_sign():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(5000).astype(np.float32)
    x[::7] = 0.0
    x[1::11] = -0.0
    x[2::13] = np.float32(1e-45)      # smallest subnormal
    x[3::13] = np.float32(-1e-45)
    q, _, _ = oracle.quantize(x, 1)
    np.testing.assert_array_equal(q, np.sign(x).astype(np.int8))


def test_quantize_special_values():
    x = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 1e-45, -1e-45], dtype=np.float32)
    q1, nf1, _ = oracle.quantize(x, 1)
    assert q1.tolist() == [0, 0, 1, -1, 0, 0, 1, -1] and nf1 == 4
    q8, nf8, _ = oracle.quantize(x, 8, 2.0)
    assert q8.tolist() == [0, 0, 127, -127, 0, 0, 0, 0] and nf8 == 4
    qz, _, _ = oracle.quantize(np.array([1.0, -3.0], np.float32), 4, None)
    assert qz.tolist() != [0, 0]


@pytest.mark.parametrize("bits", [2, 4, 8])
def test_quantize_thresholds_monotone_odd(bits):
    """phi(0)=0, odd symmetry, monotone, and the exact cell edges at (k+1/2)/s.
    With s = 1/2 the product x*s is exact, so the edge of cell k is x = 2k+1:
    the float just below maps to k, just above to k+1, the edge itself rounds
    half to even."""
    K = oracle.kmax(bits)
    s = 0.5
    xs = []
    for k in range(K):
        e = np.float32(2 * k + 1)
        xs += [np.nextafter(e, np.float32(-np.inf)), e, np.nextafter(e, np.float32(np.inf))]
    xs = np.array(xs, dtype=np.float32)
    q, _, _ = oracle.quantize(xs, bits, s)
    for k in range(K):
        lo, at, hi = q[3 * k:3 * k + 3]
        assert lo == k and hi == k + 1
        assert at == (k if k % 2 == 0 else k + 1)       # ties to even
    big = np.array([2 * K + 1, 1e30, np.float32(3.4e38)], dtype=np.float32)
    assert oracle.quantize(big, bits, s)[0].tolist() == [K, K, K]
    rng = np.random.default_rng(5)
    x = np.sort((rng.standard_normal(4000) * 4).astype(np.float32))
    qs, _, _ = oracle.quantize(x, bits, 0.8125)
    assert np.all(np.diff(qs.astype(np.int64)) >= 0)
    qn, _, _ = oracle.quantize(-x, bits, 0.8125)
    np.testing.assert_array_equal(qn, -qs)
    assert oracle.quantize(np.zeros(3, np.float32), bits, 0.8125)[0].tolist() == [0, 0, 0]


# ------------------------------------------------------------------ scale --

def test_sumsq_exactly_rounded_hand_derived():
    """Squares [2^54, 1 x k]: the exact sum is 2^54 + k, and ulp(2^54) = 4.
    Rounded once to nearest (ties to even): k = 7 -> 2^54 + 8; k = 6 is a tie
    between 2^54 + 4 (odd significand) and 2^54 + 8 (even) -> 2^54 + 8; k = 5
    -> 2^54 + 4. A pairwise tree over [2^54, 1 x 7] would give 2^54 + 4 and a
    left-to-right sum 2^54."""
    for k, want in ((7, 2.0 ** 54 + 8), (6, 2.0 ** 54 + 8), (5, 2.0 ** 54 + 4), (1, 2.0 ** 54)):
        x = np.array([2.0 ** 27] + [1.0] * k, dtype=np.float32)
        assert oracle.sumsq(x) == want
        assert oracle.sumsq(x[::-1]) == want
    assert oracle.sumsq(np.array([3.0], np.float32)) == 9.0
    assert oracle.sumsq(np.array([1.0, 2.0, 3.0], np.float32)) == 14.0


def test_sumsq_equals_exact_rational_and_ignores_order():
    """S equals the exact rational sum of the squares rounded once
    (Fraction arithmetic, float() rounds correctly), for data spanning many
    binades, and is unchanged by any permutation of the samples; non-finite
    samples add nothing."""
    rng = np.random.default_rng(2)
    for n in (1, 5, 255, 1000, 4099):
        x = (rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n))).astype(np.float32)
        exact = sum((Fraction(float(v)) ** 2 for v in x), Fraction(0))
        assert oracle.sumsq(x) == float(exact)
        for _ in range(3):
            assert oracle.sumsq(rng.permutation(x)) == float(exact)
    xi = rng.integers(-1000, 1001, size=65536 + 17)
    assert oracle.sumsq(xi.astype(np.float32)) == float(int((xi.astype(np.int64) ** 2).sum()))
    x = rng.standard_normal(100).astype(np.float32)
    y = x.copy()
    y[5], y[6] = np.nan, np.inf
    x[5], x[6] = 0.0, 0.0
    assert oracle.sumsq(y) == oracle.sumsq(x)
    # float32 subnormals square to normal float64 values (>= 2^-298)
    tiny = np.array([np.float32(2.0 ** -149)] * 3, np.float32)
    assert oracle.sumsq(tiny) == 3 * 2.0 ** -298


@pytest.mark.parametrize("bits", [2, 4, 8])
@pytest.mark.parametrize("c", [0.25, 1.0, 8.0])
def test_inv_step_closed_form(bits, c):
    """x = +-c: S = n c^2 exactly, sigma = c, inv_step = fl32((2K+1)/(6c))."""
    n = 1000
    x = np.full(n, c, np.float32)
    x[::2] = -c
    K = oracle.kmax(bits)
    expect = np.float32(float(Fraction(2 * K + 1) / (6 * Fraction(c))))
    assert oracle.inv_step(x, bits) == expect
    assert oracle.inv_step(np.zeros(7, np.float32), bits) == 0.0


def test_uniform_quantizer_cells_tile_three_sigma():
    """With inv_step = (2K+1)/(6 sigma), the cell of code K starts at
    (K - 1/2) step and the outer edge (K + 1/2) step equals 3 sigma."""
    for bits in (2, 4, 8):
        K = oracle.kmax(bits)
        step = Fraction(6, 2 * K + 1)          # sigma = 1
        assert (K + Fraction(1, 2)) * step == 3


# --------------------------------------------------------------- Theorem 1 --

def _exact_shift_pair(rng, n, d, a):
    """Untruncated support: x has its non-zeros inside a window that stays in
    [0, n) after the shift, so x[m] = a y[m + d] holds for every m (Eq. (2))."""
    L = n - abs(d)
    s = rng.standard_normal(L)
    x = np.zeros(n)
    y = np.zeros(n)
    x0 = max(0, -d)
    x[x0:x0 + L] = s
    y[x0 + d:x0 + d + L] = s / a
    return x.astype(np.float32), y.astype(np.float32)


def _monotone_map(rng, kind, k):
    if kind == "sign":
        return lambda z: np.sign(z).astype(np.int64)
    if kind == "thresholds":
        pos = np.sort(rng.exponential(1.0, size=k))
        neg = np.sort(rng.exponential(1.0, size=k))
        return lambda z: (np.searchsorted(pos, np.maximum(z, 0), side="right")
                          - np.searchsorted(neg, np.maximum(-z, 0), side="right")).astype(np.int64)
    if kind == "cubic":
        return lambda z: np.trunc(np.clip(z, -3, 3) ** 3 * k / 27).astype(np.int64)
    raise ValueError(kind)


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 10 ** 6), n=st.integers(8, 300), kind=st.sampled_from(["sign", "thresholds", "cubic"]),
       k=st.integers(1, 20))
def test_theorem1_peak_invariance(seed, n, kind, k):
    """Theorem 1: for monotone phi, psi with phi(0)=psi(0)=0 the integer
    correlation attains its maximum at the true shift nu."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(-(n // 2), n // 2 + 1))
    a = float(rng.uniform(0.2, 5.0))
    x, y = _exact_shift_pair(rng, n, d, a)
    phi, psi = _monotone_map(rng, kind, k), _monotone_map(rng, kind, k)
    u, v = phi(x.astype(np.float64)), psi(y.astype(np.float64))
    assert phi(np.zeros(1))[0] == 0 and psi(np.zeros(1))[0] == 0
    r = oracle.xcorr(u.astype(np.int8), v.astype(np.int8), -(n - 1), n - 1)
    lag, rmax, nt = oracle.argmax(r, -(n - 1))
    assert r[d + n - 1] == rmax
    assert lag <= d
    if nt == 1:
        assert lag == d


@pytest.mark.parametrize("bits", [1, 2, 4, 8])
def test_algorithm1_refined_returns_true_shift(bits):
    """Algorithm 1 with its tie-refinement step: ties are resolved by x * y, which is strictly
    maximal at nu on exact shifts (Cauchy-Schwarz), so the set is {nu}."""
    rng = np.random.default_rng(100 + bits)
    for _ in range(20):
        n = int(rng.integers(16, 400))
        d = int(rng.integers(-(n // 2), n // 2 + 1))
        x, y = _exact_shift_pair(rng, n, d, float(rng.uniform(0.5, 2.0)))
        res = oracle.estimate_refined(x, y, bits, -(n - 1), n - 1)
        assert res["lag_set"] == [d]
        assert res["r"][d + n - 1] == res["rmax"]


# ---------------------------------------------------------- float64 xcorr --

def test_xcorr_f64_matches_numpy_within_rounding():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(700).astype(np.float32)
    y = rng.standard_normal(500).astype(np.float32)
    lags = np.arange(-699, 500)
    r = oracle.xcorr_f64_at(x, y, lags)
    ref = np.correlate(y.astype(np.float64), x.astype(np.float64), "full")
    scale = np.correlate(np.abs(y).astype(np.float64), np.abs(x).astype(np.float64), "full")
    assert np.all(np.abs(r - ref) <= 700 * np.finfo(np.float64).eps * scale + 1e-300)


def test_xcorr_f64_peak_at_exact_shift():
    rng = np.random.default_rng(10)
    x, y = _exact_shift_pair(rng, 300, 37, 1.5)
    lags = np.arange(-299, 300)
    r = oracle.xcorr_f64_at(x, y, lags)
    assert lags[int(np.argmax(r))] == 37


# ------------------------------------------------------ long-signal route --

@pytest.mark.parametrize("n,k", [(4096, 127), (20000, 7)])
def test_certified_fft_route_equals_direct(n, k):
    rng = np.random.default_rng(n)
    u, v = rand_q(rng, n, k), rand_q(rng, n - 5, k)
    direct = oracle.xcorr(u, v, -(n - 1), n - 6)
    got = oracle.xcorr_long_certified(u, v, -(n - 1), n - 6, check_lags=[-(n - 1), 0, 17])
    np.testing.assert_array_equal(got, direct)


def test_fft_route_error_within_percival_bound():
    """The float64 FFT product's error never exceeds the a-priori bound, on
    full-scale codes (the worst case for the norms) with the exact
    correlation from int64 direct sums; the bound's growth factor has the
    first-order value 3k e + (3k+1) sqrt(5) e + 3k (2e) of the theorem; and at
    the long-signal workload's largest shape (two 2^22-sample b = 8 signals,
    transform 2^23) the bound stays far below 1/2."""
    rng = np.random.default_rng(77)
    for k in (4, 10, 14):
        n = 1 << k
        nu = n // 2
        u = (rng.choice([-1, 1], nu) * 127).astype(np.int8)
        v = (rng.choice([-1, 1], n - nu) * 127).astype(np.int8)
        exact = oracle.xcorr(u, v, -(nu - 1), n - nu - 1)
        got = oracle.conv_fft_f64(u, v, n)
        err = float(np.max(np.abs(got - exact.astype(np.float64))))
        bound = oracle.fft_rounding_bound(u, v, n)
        assert err <= bound
        assert np.array_equal(np.rint(got).astype(np.int64), exact)
    e = 2.0 ** -53
    for k in (1, 10, 23):
        one = np.ones(1, np.int8)
        first = (3 * k + (3 * k + 1) * math.sqrt(5.0) + 6 * k) * e
        assert abs(oracle.fft_rounding_bound(one, one, 1 << k) / 1.01 / first - 1.0) < 1e-9
    # the long workload: ||u||_2 <= 127 sqrt(2^22) is the worst case
    worst = np.full(1 << 22, 127, np.int8)
    assert oracle.fft_rounding_bound(worst, worst, 1 << 23) < 0.05


# ------------------------------------------------- learned proposer (CNN) --

from oracle import cnn  # noqa: E402

TINY = cnn.Shape(ld=64, c=3, layers=2, nbins=8)


def _tiny_params(rng, s=TINY, scale=0.4):
    p = {}
    for name, sh in cnn.param_sizes(s):
        p[name] = rng.standard_normal(sh) * scale if sh else 0.7
    return p


def test_cnn_gradients_match_central_differences():
    """Every parameter's gradient of the softmax cross-entropy equals the
    central finite difference of the loss (float64, h = 1e-6)."""
    rng = np.random.default_rng(11)
    p = _tiny_params(rng)
    xd, yd = rng.standard_normal(TINY.ld), rng.standard_normal(TINY.ld)
    label = 5
    loss, g, _ = cnn.loss_and_grads(TINY, p, xd, yd, label)
    flat = cnn.flatten(TINY, p)
    gflat = cnn.flatten(TINY, g)
    h = 1e-6
    for i in range(flat.size):
        a, b = flat.copy(), flat.copy()
        a[i] += h
        b[i] -= h
        la, _, _ = cnn.loss_and_grads(TINY, cnn.unflatten(TINY, a), xd, yd, label)
        lb, _, _ = cnn.loss_and_grads(TINY, cnn.unflatten(TINY, b), xd, yd, label)
        fd = (la - lb) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_cnn_input_gradients_match_central_differences():
    """The gradient reaching the decimated inputs (encoder backward through
    every layer) equals finite differences too."""
    rng = np.random.default_rng(12)
    p = _tiny_params(rng)
    xd, yd = rng.standard_normal(TINY.ld), rng.standard_normal(TINY.ld)
    logits, (Fx, Fy, cx, cy, raw) = cnn.forward(TINY, p, xd, yd)
    loss, dlog = cnn.softmax_ce(logits, 2)
    dFx, dFy, _ = cnn.head_bwd(TINY, p, Fx, Fy, raw, dlog)
    gsink = {name: np.zeros(sh) if sh else 0.0 for name, sh in cnn.param_sizes(TINY)}
    dx = cnn.encoder_bwd(TINY, p, cx, dFx, gsink)[0]
    h = 1e-6
    for i in range(0, TINY.ld, 7):
        a, b = xd.copy(), xd.copy()
        a[i] += h
        b[i] -= h
        la = cnn.softmax_ce(cnn.forward(TINY, p, a, yd)[0], 2)[0]
        lb = cnn.softmax_ce(cnn.forward(TINY, p, b, yd)[0], 2)[0]
        assert abs((la - lb) / (2 * h) - dx[i]) <= 1e-6 * max(1.0, abs(dx[i]))


def test_cnn_zero_weights_give_uniform_logits():
    s = cnn.Shape(ld=256, c=4, layers=3, nbins=16)
    p = {name: np.zeros(sh) if sh else 1.0 for name, sh in cnn.param_sizes(s)}
    rng = np.random.default_rng(0)
    logits, _ = cnn.forward(s, p, rng.standard_normal(256), rng.standard_normal(256))
    assert np.all(logits == 0.0)
    loss, g = cnn.softmax_ce(logits, 3)
    assert abs(loss - np.log(16)) < 1e-12 and abs(g.sum()) < 1e-12


def test_cnn_single_channel_conv_is_numpy_correlate():
    """One input and one output channel, no bias: the layer is the 'same'
    correlation of numpy with the 9-tap kernel."""
    rng = np.random.default_rng(1)
    x, w = rng.standard_normal(50), rng.standard_normal(9)
    z = cnn.conv_fwd(x[None, :], w[None, None, :], np.zeros(1))[0]
    np.testing.assert_allclose(z, np.correlate(x, w, "same"), rtol=0, atol=1e-12)
    a, pooled = cnn.relu_pool_fwd(np.array([[-1.0, 3.0, 2.0, 4.0, -5.0, -6.0]]))
    assert pooled.tolist() == [[1.5, 3.0, 0.0]]


def test_cnn_head_is_channel_sum_of_numpy_correlations():
    rng = np.random.default_rng(2)
    s = cnn.Shape(ld=160, c=5, layers=2, nbins=20)
    Fx, Fy = rng.standard_normal((5, 40)), rng.standard_normal((5, 40))
    raw = cnn.head_raw(s, Fx, Fy)
    full = sum(np.correlate(Fy[c], Fx[c], "full") for c in range(5))   # index j <-> shift j - (F - 1)
    for k in range(20):
        assert abs(raw[k] - full[k - 10 + 39]) < 1e-10


def test_cnn_adam_first_step_is_signed_lr():
    """After one step, bias correction makes m_hat = g and v_hat = g^2, so the
    update is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    w1, m, v = cnn.adam_step(w, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_cnn_bins_and_bf16_rounding():
    assert cnn.label_of_lag(-65536, 512, 256) == 0
    assert cnn.label_of_lag(-65281, 512, 256) == 0
    assert cnn.label_of_lag(-65280, 512, 256) == 1
    assert cnn.label_of_lag(0, 512, 256) == 256
    assert cnn.label_of_lag(65535, 512, 256) == 511
    assert cnn.label_of_lag(10 ** 6, 512, 256) == 511
    # bfloat16 keeps 8 significant bits; ties go to the even mantissa
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -2.5])
    assert cnn.bf16_round(vals).tolist() == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5]
    top, margin = cnn.topk_margin(np.array([0.5, 2.0, 2.0, -1.0, 1.0]), 2)
    assert top.tolist() == [1, 2] and margin == 1.0          # logit_(1) - logit_(3)


def _planted_real_near_tie(n=64, ta=10, tb=20):
    """x = 2^30 at m = 0 and 1 at m = 5; y = 2^30 at ta and at tb, 1 at
    ta + 5. Then (x * y)[ta] = 2^60 + 1 and (x * y)[tb] = 2^60 exactly, but
    2^60 + 1 is not a float64 (ulp(2^60) = 256): any float64 summation of the
    products gives 2^60 at both lags."""
    x = np.zeros(n, np.float32)
    y = np.zeros(n, np.float32)
    x[0], x[5] = 2.0 ** 30, 1.0
    y[ta], y[tb], y[ta + 5] = 2.0 ** 30, 2.0 ** 30, 1.0
    return x, y


def test_exact_real_comparison_pins():
    """compare_real_xcorr is the sign of the exact difference: it separates a
    planted pair of lags that no float64 summation order separates, agrees
    with exact Fraction arithmetic on random data, is antisymmetric, and
    refine_ties keeps exactly the lags with the largest exact value."""
    x, y = _planted_real_near_tie()
    assert oracle.xcorr_f64_at(x, y, [10])[0] == oracle.xcorr_f64_at(x, y, [20])[0] == 2.0 ** 60
    assert oracle.compare_real_xcorr(x, y, 10, 20) == 1
    assert oracle.compare_real_xcorr(x, y, 20, 10) == -1
    assert oracle.refine_ties(x, y, [10, 20]) == ([10], True)
    # a third lag with the same exact value as lag 10: x[0] y[30] + x[5] y[35]
    y[30], y[35] = 2.0 ** 30, 1.0
    assert oracle.compare_real_xcorr(x, y, 30, 10) == 0
    assert oracle.refine_ties(x, y, [10, 20, 30]) == ([10, 30], True)
    rng = np.random.default_rng(21)
    xf = (rng.standard_normal(300) * np.exp2(rng.integers(-20, 20, 300))).astype(np.float32)
    yf = (rng.standard_normal(280) * np.exp2(rng.integers(-20, 20, 280))).astype(np.float32)

    def exact(tau):
        lo, hi = max(0, -tau), min(300, 280 - tau)
        return sum((Fraction(float(xf[m])) * Fraction(float(yf[m + tau])) for m in range(lo, hi)), Fraction(0))

    lags = [-299, -150, -3, 0, 1, 17, 200, 279]
    ex = {t: exact(t) for t in lags}
    for a in lags:
        assert oracle.compare_real_xcorr(xf, yf, a, a) == 0
        for b in lags:
            want = (ex[a] > ex[b]) - (ex[a] < ex[b])
            assert oracle.compare_real_xcorr(xf, yf, a, b) == want
    best = max(ex.values())
    assert oracle.refine_ties(xf, yf, lags)[0] == [t for t in lags if ex[t] == best]
    # reading for non-finite samples: a NaN or Inf inside a tied lag's
    # overlap leaves the tied set unchanged; outside every overlap it does not matter
    xn = x.copy()
    xn[7] = np.nan
    assert oracle.refine_ties(xn, y, [10, 20]) == ([10, 20], False)
    assert oracle.refine_ties(x, y, [5]) == ([5], True)
    yi = y.copy()
    yi[63] = np.inf          # inside the overlap of lag 10 (m = 53)
    assert oracle.refine_ties(x, yi, [10, 20]) == ([10, 20], False)
    yj = np.concatenate([y, [np.inf]]).astype(np.float32)   # y[64]: inside lag 10's overlap (m = 54)
    assert oracle.refine_ties(x, yj, [10, 20])[1] is False
    assert oracle.refine_ties(x[:40], yj, [10, 20]) == ([10], True)   # m + 20 < 60: y[64] is outside both overlaps


def test_estimate_refined_partial_and_planted():
    """estimate_refined on the planted near-tie plus y[25] = 2^-10: the sign
    codes' correlation ties at lags 10, 15 and 20 (value 2), the exact real
    correlation is 2^60 + 1 at lag 10, 2^31 at 15 and 2^60 + 2^-10 at 20, so
    the refined set is {10}; max_ties cuts the tied list to its smallest lags."""
    x, y = _planted_real_near_tie()
    y[25] = 2.0 ** -10
    res = oracle.estimate_refined(x, y, 1, 0, 40)
    tied = (np.nonzero(res["r"] == res["rmax"])[0]).tolist()
    assert 10 in tied and 20 in tied and res["n_ties"] == len(tied) >= 2
    assert res["lag_set"] == [10] and res["refined"] and not res["partial"]
    cut = oracle.estimate_refined(x, y, 1, 0, 40, max_ties=1 + tied.index(10))
    assert cut["partial"] == (len(tied) > 1 + tied.index(10))


# ---------------------------------------------------------- streaming -------
# oracle.stream cuts the correlation of the whole stream into the lags each
# push makes final. Pinned against an overlap-save computation written out
# in plain Python loops (history of nx - 1 codes, zeros before the stream and
# after its end), with its own running argmax.

def _overlap_save_loops(u, blocks_codes):
    nx = len(u)
    hist = [0] * (nx - 1)
    t, recs = 0, []
    best = None          # (value, lag, count)
    for codes in list(blocks_codes) + [None]:
        new = [0] * (nx - 1) if codes is None else [int(c) for c in codes]
        buf = hist + new
        base = t - (nx - 1)
        r = []
        for tp in range(len(new)):
            r.append(sum(int(u[m]) * buf[m + tp] for m in range(nx)))
        blk = None
        for i, val in enumerate(r):
            lag = base + i
            if blk is None or val > blk[0]:
                blk = [val, lag, 1]
            elif val == blk[0]:
                blk[2] += 1
            if best is None or val > best[0]:
                best = [val, lag, 1]
            elif val == best[0]:
                best[2] += 1
        recs.append((base, base + len(new) - 1, r, None if blk is None else (blk[1], blk[0], blk[2]),
                     (best[1], best[0], best[2])))
        hist = buf[len(buf) - (nx - 1):] if nx > 1 else []
        if codes is not None:
            t += len(codes)
    return recs


@pytest.mark.parametrize("seed", range(8))
def test_stream_equals_overlap_save_loops(seed):
    rng = np.random.default_rng(seed)
    nx = int(rng.integers(1, 12))
    bits = [1, 2, 4, 8][seed % 4]
    x = rng.standard_normal(nx).astype(np.float32)
    sizes = [int(s) for s in rng.integers(1, 15, int(rng.integers(1, 6)))]
    blocks = [rng.standard_normal(n).astype(np.float32) for n in sizes]
    o = oracle.stream(x, blocks, bits, inv_step_y=1.7)
    v = o["v"]
    cuts = np.cumsum([0] + sizes)
    ref = _overlap_save_loops(o["u"], [v[cuts[i]:cuts[i + 1]] for i in range(len(sizes))])
    assert len(ref) == len(o["records"]) == len(sizes) + 1
    for rec, (a, b, r, blk, run) in zip(o["records"], ref):
        assert (rec["lag_lo"], rec["lag_hi"]) == (a, b)
        assert rec["r"].tolist() == r
        assert rec["block"] == blk
        assert rec["running"] == run
    # the quantized stream is the quantization of the concatenation (one map)
    q, _, _ = oracle.quantize(np.concatenate(blocks), bits, 1.7)
    assert np.array_equal(q, v)


def test_stream_running_argmax_ties_across_blocks():
    """A one-sample template makes r the stream codes themselves: equal maxima
    in the first and third blocks give one running maximiser set of size 2
    that starts at the earlier lag."""
    x = np.array([1.0], np.float32)
    blocks = [np.array([0.5, 3.0, -1.0], np.float32), np.array([1.0], np.float32),
              np.array([-2.0, 3.0, 0.0, 3.0], np.float32)]
    o = oracle.stream(x, blocks, 8, inv_step_y=10.0)
    recs = o["records"]
    assert recs[0]["running"][0] == 1 and recs[0]["running"][2] == 1
    assert recs[2]["block"] == (5, recs[0]["running"][1], 2)
    assert recs[2]["running"] == (1, recs[0]["running"][1], 3)
    assert recs[3]["r"].size == 0 and recs[3]["block"] is None


# ------------------------------------------------ non-uniform quantizers ----

def test_lloyd_max_gauss_matches_max_1960_tables():
    """Lloyd-Max quantizers of a unit Gaussian as tabulated by J. Max,
    'Quantizing for minimum distortion' (1960): 3 levels, boundary 0.6120 and
    level 1.2240; 7 levels, boundaries 0.2803, 0.8744, 1.611 and levels 0.5606,
    1.188, 2.033."""
    t, y = oracle.lloyd_max_gauss(1)
    assert abs(t[0] - 0.6120) < 5e-5 and abs(y[0] - 1.2240) < 5e-5
    t, y = oracle.lloyd_max_gauss(3)
    np.testing.assert_allclose(t, [0.2803, 0.8744, 1.611], atol=6e-4)
    np.testing.assert_allclose(y, [0.5606, 1.188, 2.033], atol=6e-4)


@pytest.mark.parametrize("K", [1, 3, 7])
def test_lloyd_max_gauss_is_a_fixed_point(K):
    """Boundaries are midpoints of neighbouring levels and levels are the
    conditional means of their cells (Gaussian pdf/cdf from math.erf)."""
    t, y = oracle.lloyd_max_gauss(K)
    lv = np.concatenate([[0.0], y])
    np.testing.assert_allclose(t, (lv[:-1] + lv[1:]) / 2, rtol=0, atol=1e-14)
    pdf = lambda a: math.exp(-a * a / 2) / math.sqrt(2 * math.pi)
    cdf = lambda a: 0.5 * (1 + math.erf(a / math.sqrt(2)))
    for k in range(K):
        a = t[k]
        b = t[k + 1] if k + 1 < K else math.inf
        num = pdf(a) - (pdf(b) if b != math.inf else 0.0)
        den = (cdf(b) if b != math.inf else 1.0) - cdf(a)
        assert abs(y[k] - num / den) < 1e-12
    assert np.all(np.diff(t) > 0) and t[0] > 0


@pytest.mark.parametrize("K", [1, 7])
def test_mulaw_boundaries_closed_form_and_uniform_limit(K):
    t = oracle.mulaw_thresholds(K)
    comp = np.log1p(255.0 * t / 3.0) / np.log1p(255.0)
    np.testing.assert_allclose(comp, (np.arange(1, K + 1) - 0.5) / (K + 0.5), atol=1e-14)
    # mu -> 0: the compressor is the identity, the cells those of the uniform quantizer
    tu = oracle.mulaw_thresholds(K, mu=1e-9) * (2 * K + 1) / 6.0
    np.testing.assert_allclose(tu, np.arange(1, K + 1) - 0.5, atol=1e-6)


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("bits", [2, 4])
def test_nonuniform_quantize_counts_boundaries(kind, bits):
    """Codes equal the number of float32 boundaries strictly below |z|, signed,
    with z the float32 product x * inv_step (checked sample by sample); the map
    is odd, monotone and fixes 0; NaN -> 0, +-Inf -> +-K."""
    rng = np.random.default_rng(kind * 10 + bits)
    x = (rng.standard_normal(400) * 1.3).astype(np.float32)
    x[:4] = [0.0, -0.0, np.nan, np.inf]
    x[4] = -np.inf
    q, nf, s = oracle.quantize_nonuniform(x, bits, kind)
    T = oracle.nonuniform_table(kind, bits)
    K = oracle.kmax(bits)
    assert nf == 3 and q[0] == 0 and q[1] == 0 and q[2] == 0 and q[3] == K and q[4] == -K
    for i in range(5, x.size):
        z = np.float32(x[i]) * np.float32(s)
        c = sum(1 for t in T if abs(float(z)) > float(t))
        assert q[i] == (c if z > 0 else -c)
    srt = np.sort(x[5:])
    qs, _, _ = oracle.quantize_nonuniform(srt, bits, kind, s)
    assert np.all(np.diff(qs.astype(int)) >= 0)
    qn, _, _ = oracle.quantize_nonuniform(-x[5:], bits, kind, s)
    np.testing.assert_array_equal(qn, -q[5:])
    assert np.all(np.abs(q) <= K)
    np.testing.assert_array_equal(oracle.quantize_nonuniform(x, bits, 0)[0], oracle.quantize(x, bits)[0])
