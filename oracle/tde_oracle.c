/*
 * CPU oracle for the exact integer time-difference estimator.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do. It shares no code, header or table with the HIP library.
 *
 * Everything here is the plain definition written out, in the order the paper
 * states it, with no blocking or reordering:
 *   - the cross-correlation (x * y)[n] = sum_m x[m] y[m+n] of two finite-length
 *     sequences (Section 2.2, Eq. (1));
 *   - Algorithm 1, quantization step: integer-valued monotone maps phi, psi with
 *     phi(0) = psi(0) = 0 (sign with sign(0) = 0 as in Section 4.2, or a
 *     symmetric mid-tread uniform quantizer on [-3 sigma, 3 sigma]);
 *   - Algorithm 1, correlation step: w = u * v, accumulated in int64;
 *   - Algorithm 1, argmax step: the argmax set, reported as its smallest element,
 *     the maximum and the size of the set (Remark 1: ties are legitimate).
 *   - the real-valued correlation of the unquantized signals in float64,
 *     summed in ascending m (lag accuracy of the real correlation);
 *   - a plain radix-2 complex FFT (Cooley-Tukey, decimation in time) used to
 *     correlate long integer sequences in float64; its rounding error is
 *     bounded a priori (Percival's bound for FFT-based products), so the
 *     rounded result is exact whenever that bound is below 1/2.
 *
 * Plain C, compiled without fast-math: every float operation below is one
 * correctly rounded IEEE-754 operation.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ---------------------------------------------------------------- scale -- */

/* Largest code magnitude K of a b-bit symmetric quantizer; sign (b = 1) is
 * ternary with K = 1 (Section 4.2 uses sign with sign(0) = 0, i.e. K = 1). */
int oracle_kmax(int bits) {
    if (bits == 1) return 1;
    return (1 << (bits - 1)) - 1;
}

/* inv_step of the uniform quantizer on [-3 sigma, 3 sigma] with 2K+1 cells:
 * step = 6 sigma / (2K+1), sigma = sqrt(S / n). Zero when S is zero. */
float oracle_inv_step_from_sumsq(double S, int64_t n, int bits) {
    if (!(S > 0.0)) return 0.0f;
    int K = oracle_kmax(bits);
    double var = S / (double)n;
    double sigma = sqrt(var);
    double inv = (double)(2 * K + 1) / (6.0 * sigma);
    return (float)inv;
}

/* ------------------------------------------------------------- quantize -- */

static uint32_t f32_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/* Algorithm 1, quantization step. Returns the number of non-finite samples.
 * bits == 1: sign from the IEEE bits: +1 for positive non-zero (including
 *   +Inf), -1 for negative non-zero (including -Inf), 0 for +-0 and NaN.
 * bits in {2,4,8}: K = 2^(b-1)-1, t = fl32(x * inv_step), q = clamp(rne(t),
 *   -K, K); NaN maps to 0; inv_step == 0 maps everything to 0. */
int64_t oracle_quantize(const float* x, int64_t n, int bits, float inv_step, int8_t* q) {
    int64_t nonfinite = 0;
    int K = oracle_kmax(bits);
    for (int64_t m = 0; m < n; ++m) {
        uint32_t b = f32_bits(x[m]);
        uint32_t mag = b & 0x7fffffffu;
        int is_nan = mag > 0x7f800000u;
        int is_inf = mag == 0x7f800000u;
        if (is_nan || is_inf) nonfinite++;
        int8_t out;
        if (bits == 1) {
            if (is_nan || mag == 0) out = 0;
            else out = (b >> 31) ? -1 : 1;
        } else {
            if (is_nan || inv_step == 0.0f) {
                out = 0;
            } else {
                float t = x[m] * inv_step;     /* one rounded fp32 multiply */
                float rq = rintf(t);           /* ties to even (default mode) */
                if (rq > (float)K) rq = (float)K;
                if (rq < -(float)K) rq = -(float)K;
                out = (int8_t)(int)rq;
            }
        }
        q[m] = out;
    }
    return nonfinite;
}

/* ---------------------------------------------------------- correlation -- */

/* Eq. (1) on integer sequences u on [0, nu), v on [0, nv), zero elsewhere:
 * r[i] = sum_m u[m] v[m + tau], tau = lag_lo + i, int64 accumulation. */
static int64_t xcorr_one(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int64_t tau) {
    int64_t m0 = tau < 0 ? -tau : 0;
    int64_t m1 = nu < nv - tau ? nu : nv - tau;
    int64_t acc = 0;
    for (int64_t m = m0; m < m1; ++m) acc += (int64_t)u[m] * (int64_t)v[m + tau];
    return acc;
}

void oracle_xcorr_i64(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv,
                      int64_t lag_lo, int64_t lag_hi, int64_t* r) {
    int64_t L = lag_hi - lag_lo + 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < L; ++i) r[i] = xcorr_one(u, nu, v, nv, lag_lo + i);
}

/* The same sum at an arbitrary list of lags. */
void oracle_xcorr_i64_at(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv,
                         const int64_t* lags, int64_t nlags, int64_t* r) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nlags; ++i) r[i] = xcorr_one(u, nu, v, nv, lags[i]);
}

/* Algorithm 1, argmax step over r[0..L): the maximum, the smallest maximising lag
 * and the number of maximisers. */
void oracle_argmax_i64(const int64_t* r, int64_t L, int64_t lag_lo,
                       int64_t* lag, int64_t* rmax, int64_t* nties) {
    int64_t best = r[0], at = 0, cnt = 1;
    for (int64_t i = 1; i < L; ++i) {
        if (r[i] > best) { best = r[i]; at = i; cnt = 1; }
        else if (r[i] == best) cnt++;
    }
    *lag = lag_lo + at;
    *rmax = best;
    *nties = cnt;
}

/* Eq. (1) on the unquantized float signals, in float64, summed in ascending
 * m. Used for the refinement of tied lags (Algorithm 1, tie-refinement step) and for the
 * accuracy of the plain real correlation. */
void oracle_xcorr_f64_at(const float* x, int64_t nx, const float* y, int64_t ny,
                         const int64_t* lags, int64_t nlags, double* r) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nlags; ++i) {
        int64_t tau = lags[i];
        int64_t m0 = tau < 0 ? -tau : 0;
        int64_t m1 = nx < ny - tau ? nx : ny - tau;
        double acc = 0.0;
        for (int64_t m = m0; m < m1; ++m) acc += (double)x[m] * (double)y[m + tau];
        r[i] = acc;
    }
}

/* ------------------------------------------------------------ long FFT -- */

/* Twiddles w_j = exp(-2 pi i j / n), j < n/2, evaluated in long double (x86
 * extended precision, 64-bit significand) and rounded once to double: each
 * is within about one unit roundoff of double of the exact value (the bound
 * takes beta = 2 eps). The inverse transform uses their conjugates. */
static void fft_twiddles(int64_t n, double* twr, double* twi) {
    for (int64_t j = 0; j < n / 2; ++j) {
        long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)n;
        twr[j] = (double)cosl(a);
        twi[j] = (double)sinl(a);
    }
}

/* In-place radix-2 decimation-in-time complex FFT of length n = 2^k (re, im
 * separate arrays); inverse = 1 conjugates the twiddles (unscaled inverse).
 * Every butterfly is t = w b (four real products, two sums, each rounded
 * once), then a + t and a - t: the arithmetic Percival's error bound
 * describes. */
static void fft_r2(double* re, double* im, int64_t n, int inverse, const double* twr, const double* twi) {
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len / 2, step = n / len;
#pragma omp parallel for schedule(static) if (n >= 65536)
        for (int64_t b = 0; b < n; b += len) {
            for (int64_t k = 0; k < half; ++k) {
                double wr = twr[k * step], wi = inverse ? -twi[k * step] : twi[k * step];
                double br = re[b + k + half], bi = im[b + k + half];
                double tr = wr * br - wi * bi;
                double ti = wr * bi + wi * br;
                double ar = re[b + k], ai = im[b + k];
                re[b + k] = ar + tr;
                im[b + k] = ai + ti;
                re[b + k + half] = ar - tr;
                im[b + k + half] = ai - ti;
            }
        }
    }
}

/* Linear convolution c = rev(u) conv v of int8 sequences (length nu + nv - 1)
 * through complex FFTs of length n >= nu + nv - 1 (a power of two), in
 * float64, unrounded: out[j] approximates r[j - (nu - 1)] of Eq. (1).
 * scratch: 5 n doubles (two complex arrays and the twiddles). */
void oracle_conv_fft(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int64_t n, double* out,
                     double* scratch) {
    double *ar = scratch, *ai = scratch + n, *br = scratch + 2 * n, *bi = scratch + 3 * n;
    double *twr = scratch + 4 * n, *twi = scratch + 4 * n + n / 2;
    for (int64_t i = 0; i < n; ++i) {
        ar[i] = i < nu ? (double)u[nu - 1 - i] : 0.0;
        br[i] = i < nv ? (double)v[i] : 0.0;
        ai[i] = 0.0;
        bi[i] = 0.0;
    }
    fft_twiddles(n, twr, twi);
    fft_r2(ar, ai, n, 0, twr, twi);
    fft_r2(br, bi, n, 0, twr, twi);
    for (int64_t i = 0; i < n; ++i) {      /* pointwise complex product */
        double pr = ar[i] * br[i] - ai[i] * bi[i];
        double pi = ar[i] * bi[i] + ai[i] * br[i];
        ar[i] = pr;
        ai[i] = pi;
    }
    fft_r2(ar, ai, n, 1, twr, twi);
    double inv_n = 1.0 / (double)n;        /* a power of two: exact */
    for (int64_t j = 0; j < nu + nv - 1; ++j) out[j] = ar[j] * inv_n;
}

/* Number of OpenMP threads the direct sums use. */
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }

/* Threads for the later direct sums (the CPU baseline times one thread too). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
