"""Seeded synthetic signal pairs for the time-difference workloads.

This module only draws signals: it holds none of the estimator's arithmetic
(no quantization, correlation or argmax). Both the HIP path and the CPU oracle
are fed the same float32 bytes produced here.

Conventions (Section 2.2, Eqs. (1)-(2)): the correlation is
(x * y)[tau] = sum_m x[m] y[m + tau], so for y = x delayed by d,
y[n] = x[n - d], the peak sits at tau = +d. Delays use zero fill: y[n] = 0 where
n - d falls outside [0, N). Noise is added to y only, at a signal-to-noise
ratio measured as mean square of the clean delayed signal over its non-zero
support against the noise variance (the paper's squared l2 norm per unit
time, Section 4.2).

Every generator takes a ``numpy.random.Generator``; ``pair_rngs`` spawns one
per pair from ``SeedSequence(2509_19974 + config)``. Signals are drawn in
float64 and cast to float32 once.
"""
from __future__ import annotations

import numpy as np
from scipy import signal as _sig

BASE_SEED = 2509_19974


def pair_rngs(config: int, npairs: int, salt: int = 0):
    ss = np.random.SeedSequence(BASE_SEED + config + 1000 * salt)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(npairs)]


# ---------------------------------------------------------------- sources --

def white(rng, n: int) -> np.ndarray:
    return rng.standard_normal(n)


def ar1(rng, n: int, coef: float = 0.9, burn: int = 4096) -> np.ndarray:
    e = rng.standard_normal(n + burn)
    return _sig.lfilter([1.0], [1.0, -coef], e)[burn:]


def ar2(rng, n: int, p1: float = 0.95, p2: float = 0.6, burn: int = 4096) -> np.ndarray:
    """AR(2) with real poles p1, p2: s[n] = (p1+p2) s[n-1] - p1 p2 s[n-2] + e[n]."""
    e = rng.standard_normal(n + burn)
    return _sig.lfilter([1.0], [1.0, -(p1 + p2), p1 * p2], e)[burn:]


def exp_decay_response(rng, taps: int, decay: float) -> np.ndarray:
    """h[k] = g[k] exp(-k / decay), g ~ N(0,1), unit energy."""
    k = np.arange(taps, dtype=np.float64)
    h = rng.standard_normal(taps) * np.exp(-k / decay)
    return h / np.sqrt(np.dot(h, h))


def reverb_response(rng, t60: int) -> np.ndarray:
    """Random response of length T with a 60 dB decay over T samples:
    h[k] = g[k] 10^(-3k/T), unit energy."""
    k = np.arange(t60, dtype=np.float64)
    h = rng.standard_normal(t60) * 10.0 ** (-3.0 * k / t60)
    return h / np.sqrt(np.dot(h, h))


def filtered_noise(rng, n: int, h: np.ndarray) -> np.ndarray:
    """Steady-state white noise filtered by h (no start-up transient)."""
    e = rng.standard_normal(n + h.size - 1)
    return _sig.fftconvolve(e, h, mode="valid")


# ------------------------------------------------------------------ pairs --

def delay_zero_fill(x: np.ndarray, d: int, ny: int | None = None) -> np.ndarray:
    """y[n] = x[n - d] for 0 <= n - d < len(x), else 0; length ny (default len(x))."""
    n = x.size if ny is None else ny
    y = np.zeros(n, dtype=np.float64)
    lo = max(0, d)
    hi = min(n, x.size + d)
    if hi > lo:
        y[lo:hi] = x[lo - d:hi - d]
    return y


def add_noise(rng, clean: np.ndarray, snr_db: float) -> np.ndarray:
    nz = clean != 0
    ps = float(np.mean(clean[nz] ** 2)) if nz.any() else 0.0
    sd = np.sqrt(ps / 10.0 ** (snr_db / 10.0))
    return clean + sd * rng.standard_normal(clean.size)


def make_pair(rng, x: np.ndarray, d: int, snr_db: float | None):
    y = delay_zero_fill(x, d)
    if snr_db is not None:
        y = add_noise(rng, y, snr_db)
    return x.astype(np.float32), y.astype(np.float32)


# ---------------------------------------------------------------- configs --
# Each returns a list of dicts: x, y (float32), d (true delay), bits,
# lag_lo, lag_hi, plus the drawing parameters.

def config1_single(npairs: int = 1, n: int = 4096, salt: int = 0):
    """Single pair: white noise, d ~ U{-512..512}, zero fill, 20 dB on y,
    sign quantization, lags [-1024, 1024]."""
    out = []
    for rng in pair_rngs(1, npairs, salt):
        x = white(rng, n)
        d = int(rng.integers(-512, 513))
        xf, yf = make_pair(rng, x, d, 20.0)
        out.append(dict(x=xf, y=yf, d=d, bits=1, lag_lo=-1024, lag_hi=1024, snr_db=20.0))
    return out


def config2_batch(bits: int, npairs: int = 64, n: int = 65536, salt: int = 0):
    """AR(2) coloured noise (poles 0.95, 0.6), d ~ U{-n/4..n/4}, SNR ~ U[0,30]
    dB on y, uniform quantizer with the given bits, full lag range."""
    out = []
    for rng in pair_rngs(2, npairs, salt):
        x = ar2(rng, n)
        d = int(rng.integers(-(n // 4), n // 4 + 1))
        snr = float(rng.uniform(0.0, 30.0))
        xf, yf = make_pair(rng, x, d, snr)
        out.append(dict(x=xf, y=yf, d=d, bits=bits, lag_lo=-(n - 1), lag_hi=n - 1, snr_db=snr))
    return out


def config3_long(n: int, npairs: int = 8, salt: int = 0):
    """Gaussian noise through a random exponentially decaying response (decay
    4800 samples, 8192 taps), d ~ U{-n/2..n/2}, noiseless zero-fill shift,
    b = 8, full lag range."""
    out = []
    for rng in pair_rngs(3, npairs, salt + n):
        h = exp_decay_response(rng, 8192, 4800.0)
        x = filtered_noise(rng, n, h)
        d = int(rng.integers(-(n // 2), n // 2 + 1))
        xf, yf = make_pair(rng, x, d, None)
        out.append(dict(x=xf, y=yf, d=d, bits=8, lag_lo=-(n - 1), lag_hi=n - 1, snr_db=None))
    return out


def config4_uneven(npairs: int = 4096, nmin_log2: float = 10.0, nmax_log2: float = 18.0, salt: int = 0):
    """N = round(2^U[10,18]); b ~ U{1,2,4}; lags +-floor(N/4); white or AR(1)
    (0.9) with probability 1/2 each; SNR ~ U[0,30] dB; d ~ U{-floor(N/4)..}."""
    out = []
    for rng in pair_rngs(4, npairs, salt):
        n = int(round(2.0 ** rng.uniform(nmin_log2, nmax_log2)))
        bits = int(rng.choice([1, 2, 4]))
        kind = "white" if rng.random() < 0.5 else "ar1"
        x = white(rng, n) if kind == "white" else ar1(rng, n, 0.9)
        L = n // 4
        d = int(rng.integers(-L, L + 1))
        snr = float(rng.uniform(0.0, 30.0))
        xf, yf = make_pair(rng, x, d, snr)
        out.append(dict(x=xf, y=yf, d=d, bits=bits, lag_lo=-L, lag_hi=L, snr_db=snr, kind=kind))
    return out


def config5_reverb(npairs: int = 1024, n: int = 1 << 18, max_lag: int = 1 << 16, salt: int = 0,
                   t60_range=(2000, 12000)):
    """Reverberant pairs: x = white noise through a random response with a
    60 dB decay over T ~ U[2000, 12000] samples; y = x delayed by
    d ~ U{-max_lag..max_lag-1} plus noise at SNR ~ U[0,30] dB; b = 4; lags
    [-max_lag, max_lag - 1] (the union of the proposer's 256-lag bins)."""
    out = []
    for rng in pair_rngs(5, npairs, salt):
        t60 = int(rng.integers(t60_range[0], t60_range[1] + 1))
        h = reverb_response(rng, t60)
        x = filtered_noise(rng, n, h)
        d = int(rng.integers(-max_lag, max_lag))
        snr = float(rng.uniform(0.0, 30.0))
        xf, yf = make_pair(rng, x, d, snr)
        out.append(dict(x=xf, y=yf, d=d, bits=4, lag_lo=-max_lag, lag_hi=max_lag - 1, snr_db=snr, t60=t60))
    return out


def config5_reverb_torch(torch, npairs: int, salt: int = 0, n: int = 1 << 18, max_lag: int = 1 << 16,
                         device="cuda", t60_range=(2000, 12000)):
    """The reverberant recipe of ``config5_reverb`` drawn with torch's
    generator on ``device`` (float32), for training-scale sets: the host
    recipe costs tens of milliseconds per pair. Per pair: T ~ U{t60_range};
    h[k] = g[k] 10^(-3k/T) for k < T, unit energy; x = steady-state white
    noise through h (the valid part of a linear convolution, taken by FFT);
    d ~ U{-max_lag..max_lag-1}; y[n] = x[n - d] (zero fill) plus white noise
    at SNR ~ U[0, 30] dB (power of the delayed signal over its support).
    The same salt and device give the same bytes. Returns a dict of tensors
    x, y [npairs][n] float32 and d, snr_db, t60 [npairs]."""
    g = torch.Generator(device=device)
    g.manual_seed(BASE_SEED + 5 + 1000 * salt)
    tmax = int(t60_range[1])
    t60 = torch.randint(int(t60_range[0]), tmax + 1, (npairs,), generator=g, device=device)
    k = torch.arange(tmax, device=device, dtype=torch.float32)
    env = torch.pow(10.0, -3.0 * k[None, :] / t60[:, None].float()) * (k[None, :] < t60[:, None]).float()
    h = torch.randn(npairs, tmax, generator=g, device=device) * env
    h = h / torch.linalg.vector_norm(h, dim=1, keepdim=True)
    e = torch.randn(npairs, n + tmax - 1, generator=g, device=device)
    nfft = 1
    while nfft < n + 2 * tmax - 2:
        nfft *= 2
    full = torch.fft.irfft(torch.fft.rfft(e, nfft) * torch.fft.rfft(h, nfft), nfft)
    del e
    x = full[:, tmax - 1:tmax - 1 + n].contiguous()
    del full
    d = torch.randint(-max_lag, max_lag, (npairs,), generator=g, device=device)
    src = torch.arange(n, device=device)[None, :] - d[:, None]
    inside = (src >= 0) & (src < n)
    y = torch.where(inside, torch.gather(x, 1, src.clamp(0, n - 1)), torch.zeros((), device=device))
    snr = torch.rand(npairs, generator=g, device=device) * 30.0
    ps = (y * y).sum(dim=1) / inside.sum(dim=1).clamp(min=1)
    sd = torch.sqrt(ps / torch.pow(10.0, snr / 10.0))
    y = y + sd[:, None] * torch.randn(npairs, n, generator=g, device=device)
    return {"x": x, "y": y.contiguous(), "d": d, "snr_db": snr, "t60": t60}


def stream_embedded(nx: int = 8192, block: int = 65536, nblocks: int = 64, noise: float = 0.7, salt: int = 0):
    """Streaming workload: a white template of nx samples added once, at a
    uniform position, to white noise of standard deviation `noise` that is
    pushed in nblocks blocks of `block` samples. Returns (x, y, position)."""
    rng = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 6 + 1000 * salt))
    x = rng.standard_normal(nx)
    where = int(rng.integers(0, nblocks * block - nx))
    y = noise * rng.standard_normal(nblocks * block)
    y[where:where + nx] += x
    return x.astype(np.float32), y.astype(np.float32), where


def frac_delay(x: np.ndarray, frac: float, taps: int = 32) -> np.ndarray:
    """x delayed by a fraction of a sample (0 <= frac < 1): Hann-windowed sinc
    interpolation with `taps` taps, same length (zero outside)."""
    k = np.arange(-taps // 2 + 1, taps // 2 + 1)
    h = np.sinc(k - frac) * (0.5 + 0.5 * np.cos(np.pi * (k - frac) / (taps // 2 + 1)))
    y = np.convolve(x, h, mode="full")          # y[n] = sum_k x[n - k] h(k), k from -taps/2 + 1
    return y[taps // 2 - 1:taps // 2 - 1 + x.size]


def speech_like_mixtures(npairs: int, snr_db: float, n_target: int = 16000, n_mix: int = 80000,
                         max_delay: int = 64000, salt: int = 0):
    """Stand-in for the accuracy experiment of Section 4.2 (its speech and
    environmental-sound corpora are not available): a one-second 16 kHz
    'utterance' (AR(2) noise under a random syllable envelope of 2-5 raised-
    cosine bumps) and a five-second background (AR(1), coefficient 0.95); the
    target is delayed by nu ~ U[0, max_delay) samples (integer part by
    placement, fraction by windowed-sinc interpolation) and mixed into the
    background at the given SNR, measured as power per unit time of the
    target over its own support against the background's. Returns (targets,
    mixtures, nu) with float32 signals and float64 delays."""
    rngs = pair_rngs(7, npairs, salt)
    xs, ys, nus = [], [], []
    for rng in rngs:
        s = ar2(rng, n_target, 0.9, 0.5)
        env = np.zeros(n_target)
        t = np.arange(n_target)
        for _ in range(int(rng.integers(2, 6))):
            c = rng.uniform(0.1, 0.9) * n_target
            w = rng.uniform(0.04, 0.15) * n_target
            env += np.where(np.abs(t - c) < w, 0.5 + 0.5 * np.cos(np.pi * (t - c) / w), 0.0)
        target = s * env
        target /= np.sqrt(np.mean(target ** 2))
        bg = ar1(rng, n_mix, 0.95)
        nu = rng.uniform(0, max_delay)
        d = int(np.floor(nu))
        shifted = frac_delay(target, nu - d)
        p_t = np.mean(shifted ** 2)
        p_b = np.mean(bg ** 2)
        bg *= np.sqrt(p_t / p_b / 10.0 ** (snr_db / 10.0))
        mix = bg.copy()
        hi = min(n_mix, d + n_target)
        mix[d:hi] += shifted[:hi - d]
        xs.append(target.astype(np.float32))
        ys.append(mix.astype(np.float32))
        nus.append(nu)
    return xs, ys, np.array(nus)


def random_int_seq(rng, n: int, k: int, p_zero: float = 0.0) -> np.ndarray:
    """Uniform integers in [-k, k] with an optional extra share of zeros."""
    q = rng.integers(-k, k + 1, size=n)
    if p_zero > 0:
        q[rng.random(n) < p_zero] = 0
    return q.astype(np.int8)
