/* The C oracle's functions on small and edge-case inputs under
 * AddressSanitizer and UndefinedBehaviorSanitizer, with a few checks that
 * hold by definition (r over every full-linear lag sums to (sum u)(sum v);
 * the FFT route rounds to the direct sums; the argmax is the first maximum).
 * Exit status 0 when every check holds; the sanitizers abort on a fault. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_kmax(int bits);
float oracle_inv_step_from_sumsq(double S, int64_t n, int bits);
int64_t oracle_quantize(const float* x, int64_t n, int bits, float inv_step, int8_t* q);
void oracle_xcorr_i64(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int64_t lag_lo, int64_t lag_hi,
                      int64_t* r);
void oracle_xcorr_i64_at(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, const int64_t* lags,
                         int64_t nlags, int64_t* r);
void oracle_argmax_i64(const int64_t* r, int64_t L, int64_t lag_lo, int64_t* lag, int64_t* rmax, int64_t* nties);
void oracle_xcorr_f64_at(const float* x, int64_t nx, const float* y, int64_t ny, const int64_t* lags,
                         int64_t nlags, double* r);
void oracle_conv_fft(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int64_t n, double* out,
                     double* scratch);
void oracle_set_threads(int n);

static uint64_t st = 88172645463325252ull;
static double uni(void) {                      /* xorshift64, [0, 1) */
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) / 9007199254740992.0;
}

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++fails; } } while (0)

static void one_case(int64_t nu, int64_t nv, int bits) {
    float* x = malloc(sizeof(float) * (size_t)(nu > 0 ? nu : 1));
    float* y = malloc(sizeof(float) * (size_t)(nv > 0 ? nv : 1));
    int8_t* u = malloc((size_t)(nu > 0 ? nu : 1));
    int8_t* v = malloc((size_t)(nv > 0 ? nv : 1));
    double sx = 0, sy = 0;
    for (int64_t i = 0; i < nu; ++i) { x[i] = (float)(uni() * 2 - 1); sx += (double)x[i] * x[i]; }
    for (int64_t i = 0; i < nv; ++i) { y[i] = (float)(uni() * 2 - 1); sy += (double)y[i] * y[i]; }
    if (nu > 2) { x[0] = NAN; x[1] = INFINITY; x[2] = -0.0f; }
    oracle_quantize(x, nu, bits, oracle_inv_step_from_sumsq(sx, nu, bits), u);
    oracle_quantize(y, nv, bits, oracle_inv_step_from_sumsq(sy, nv, bits), v);
    const int64_t lo = -(nu - 1), hi = nv - 1, L = hi - lo + 1;
    int64_t* r = malloc(sizeof(int64_t) * (size_t)L);
    oracle_xcorr_i64(u, nu, v, nv, lo, hi, r);
    int64_t su = 0, sv = 0, sr = 0;
    for (int64_t i = 0; i < nu; ++i) su += u[i];
    for (int64_t i = 0; i < nv; ++i) sv += v[i];
    for (int64_t i = 0; i < L; ++i) sr += r[i];
    CHECK(sr == su * sv);
    int64_t lag, rmax, nt;
    oracle_argmax_i64(r, L, lo, &lag, &rmax, &nt);
    CHECK(r[lag - lo] == rmax && nt >= 1);
    for (int64_t i = 0; i < lag - lo; ++i) CHECK(r[i] < rmax);
    /* lags outside the support, and a list of lags */
    int64_t lags[6] = {lo - 3, lo, 0, hi, hi + 7, (lo + hi) / 2}, ra[6];
    double rf[6];
    oracle_xcorr_i64_at(u, nu, v, nv, lags, 6, ra);
    CHECK(ra[0] == 0 && ra[4] == 0 && ra[1] == r[0] && ra[3] == r[L - 1]);
    oracle_xcorr_f64_at(x, nu, y, nv, lags, 6, rf);
    /* FFT route */
    int64_t n = 1;
    while (n < nu + nv - 1) n *= 2;
    double* out = malloc(sizeof(double) * (size_t)(nu + nv - 1));
    double* scr = malloc(sizeof(double) * (size_t)(5 * n));
    oracle_conv_fft(u, nu, v, nv, n, out, scr);
    for (int64_t j = 0; j < nu + nv - 1; ++j) CHECK(llround(out[j]) == r[j]);
    free(x); free(y); free(u); free(v); free(r); free(out); free(scr);
}

int main(void) {
    oracle_set_threads(2);
    for (int b = 1; b <= 8; b *= 2) CHECK(oracle_kmax(b) >= 1);
    const int64_t sizes[][2] = {{1, 1}, {1, 7}, {7, 1}, {3, 3}, {64, 65}, {257, 100}, {1000, 1023}, {4097, 3}};
    const int bits[] = {1, 2, 4, 8};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s)
        for (size_t b = 0; b < 4; ++b) one_case(sizes[s][0], sizes[s][1], bits[b]);
    /* quantizer special values */
    float sp[8] = {0.0f, -0.0f, NAN, INFINITY, -INFINITY, 1e-45f, 3.4e38f, -3.4e38f};
    int8_t q[8];
    for (size_t b = 0; b < 4; ++b) {
        oracle_quantize(sp, 8, bits[b], 1.0f, q);
        oracle_quantize(sp, 8, bits[b], 0.0f, q);
        CHECK(q[0] == 0 && q[2] == 0);
    }
    printf("oracle driver: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
