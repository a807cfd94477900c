/*
 * tde.h -- exact integer time-difference estimation on AMD Instinct MI355X
 * (gfx950). C ABI of libtde.so.
 *
 * The method (Ueno, Sato, Ono, "On the Invariance of Cross-Correlation Peak
 * Positions Under Monotonic Signal Transformations, with Application to Fast
 * Time Difference Estimation"):
 *
 *   Section 2.2, Eq. (1):  (x * y)[tau] = sum_m x[m] y[m + tau]
 *   Theorem 1:             for monotone non-decreasing phi, psi with
 *                          phi(0) = psi(0) = 0, the correlation of phi(x) and
 *                          psi(y) peaks at the same tau as that of x and y when
 *                          x[m] = a y[m + nu] (Eq. (2)).
 *   Algorithm 1:           quantize both signals to integers, compute the
 *                          integer correlation exactly, take its argmax.
 *
 * Lag convention (Eqs. (1)-(2)): if y is x delayed by d samples,
 * y[n] = x[n - d], the correlation peaks at tau = +d. Output arrays hold
 * r[i] <-> tau = lag_lo + i.
 *
 * Conventions of every call:
 *  - Every call returns an int status: TDE_OK (0) or a negative TDE_ERR_*.
 *    Nothing throws, exits or aborts. tde_last_error() gives a thread-local
 *    message for the last failing call of this thread.
 *  - Array arguments are caller-owned DEVICE pointers (allocated on the
 *    context's device), unless a parameter says "host". The library never
 *    frees them and keeps none of them after the queued work has run; the
 *    caller keeps them alive until its stream passes that point.
 *  - Work is queued asynchronously on the caller's stream (a hipStream_t
 *    passed as void*; NULL is the default stream) and is deterministic:
 *    identical inputs give bit-identical outputs.
 *  - Argument validation is synchronous and happens before anything is
 *    queued. Data-dependent conditions (non-finite samples, all-zero
 *    signals) are reported through per-result flags, not the status.
 *  - Calls that need scratch memory take a caller-allocated device workspace
 *    (ws, ws_bytes) whose minimum size the matching *_workspace_size call
 *    returns; TDE_ERR_WS if it is too small. The hot calls allocate nothing.
 */
#ifndef TDE_H
#define TDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status -- */
#define TDE_OK               0
#define TDE_ERR_ARG         -1   /* invalid argument (null, size, bits, range) */
#define TDE_ERR_RANGE       -2   /* int32 result cannot hold the exact value */
#define TDE_ERR_WS          -3   /* workspace missing or too small */
#define TDE_ERR_HIP         -4   /* a HIP runtime call failed */
#define TDE_ERR_UNSUPPORTED -5   /* valid request the library does not handle */
#define TDE_ERR_IO          -6   /* file read/write failed (models) */

/* r_dtype values */
#define TDE_I32 0
#define TDE_I64 1

/* correlation engines (the autotuner picks one for TDE_PATH_AUTO) */
#define TDE_PATH_AUTO 0
#define TDE_PATH_MFMA 1          /* direct sums on the matrix cores: codes up to 3 as FP4
                                    (E2M1), up to 7 as FP6 (E2M3), else int8; all exact */
#define TDE_PATH_POPC 2          /* direct sums, bit planes (ternary codes only) */
#define TDE_PATH_NTT  3          /* number-theoretic transform, CRT to int64 */
#define TDE_PATH_MFMA_I8 4       /* TDE_PATH_MFMA with int8 operands for every code range */

/* result flags */
#define TDE_FLAG_NONFINITE_X 1   /* x held NaN or Inf samples */
#define TDE_FLAG_NONFINITE_Y 2
#define TDE_FLAG_ZERO_X      4   /* every code of x is 0 (so r is 0 everywhere) */
#define TDE_FLAG_ZERO_Y      8
#define TDE_FLAG_FALLBACK   16   /* learned mode: proposal margin too low, full search used */
#define TDE_FLAG_REFINED    32   /* tde_refine_ties chose among several maximisers */
#define TDE_FLAG_REFINE_PARTIAL 64  /* more maximisers than max_ties: the smallest max_ties were refined */
#define TDE_FLAG_SCALE_EXACT 128  /* an automatic scale needed the exact sum of squares (the float64
                                     tree sum's error bound straddled a float32 rounding boundary) */
#define TDE_FLAG_REFINE_EXACT 256 /* tde_refine_ties compared tied lags by exact sums */
#define TDE_FLAG_REFINE_NONFINITE 512  /* a tied lag's overlap held NaN or Inf: peak left unrefined */

typedef struct tde_ctx tde_ctx;

/* Algorithm 1, argmax step, reported for one pair: the smallest maximising lag,
 * the maximum, and the size of the argmax set (Remark 1: the quantized
 * correlation can have several peaks, the true shift always among them). */
typedef struct {
    int64_t lag;
    int64_t rmax;
    int32_t n_ties;
    int32_t flags;
} tde_peak;

/* Per-signal statistics written by tde_quantize (device memory). */
typedef struct {
    float   inv_step;      /* scale used (0 for bits = 1 or an all-zero signal) */
    int32_t flags;         /* TDE_FLAG_NONFINITE_X / TDE_FLAG_ZERO_X */
    int64_t n_nonfinite;   /* NaN or Inf samples */
    int64_t n_zero;        /* samples with code 0 */
    int64_t sum_q;         /* sum of codes */
    int64_t sum_q2;        /* sum of squared codes */
} tde_qstat;

/* ------------------------------------------------------------ context -- */

/* Create a context bound to HIP device `device` (it becomes current while
 * the library works). Owns pinned staging memory, captured graphs and timing
 * events. Fails with TDE_ERR_UNSUPPORTED on a device that is not gfx950. */
int  tde_create(tde_ctx** ctx, int device);
void tde_destroy(tde_ctx* ctx);
const char* tde_status_string(int status);
const char* tde_last_error(void);

/* --------------------------------------------------------- quantize -- */

/* Algorithm 1, quantization step: monotone integer maps phi with phi(0) = 0.
 *
 * x[n] (device, float32) -> q[n] (device, int8).
 *  bits = 1: sign with sign(0) = 0 (Section 4.2), decided from the IEEE bits:
 *            +1 for positive non-zero (incl. +Inf), -1 for negative non-zero
 *            (incl. -Inf), 0 for +-0 and NaN. inv_step is ignored.
 *  bits = 2, 4, 8: K = 2^(bits-1) - 1; t = fl32(x * inv_step) (one rounded
 *            float32 multiply); q = clamp(round_half_even(t), -K, K); NaN -> 0.
 *            The 2K+1 cells tile [-3 sigma, 3 sigma] when
 *            inv_step = (2K+1) / (6 sigma).
 *  inv_step <= 0 selects the automatic scale: sigma = sqrt(S / n) with S the
 *            exact sum of x^2 over the finite samples rounded once to
 *            float64 (nearest, ties to even; it depends on no summation
 *            order); inv_step = fl32((2K+1) / (6 sigma)) in float64
 *            operations, or 0 when S = 0 (then every code is 0). The scale
 *            used is written to stat->inv_step. The library adds the squares
 *            in float64 and forms the exact sum only when that sum's error
 *            bound leaves inv_step undecided (stat->flags then carries
 *            TDE_FLAG_SCALE_EXACT).
 *  stat (device, may be NULL) receives the tde_qstat of the signal.
 * Errors: TDE_ERR_ARG for n < 1, a null x/q, bits not in {1,2,4,8}, or a
 * non-finite inv_step; TDE_ERR_UNSUPPORTED for the automatic scale of
 * n >= 2^32 samples. ws: tde_quantize_workspace_size(n) bytes (may be 0
 * when inv_step > 0 and stat is NULL). */
size_t tde_quantize_workspace_size(int64_t n);
int tde_quantize(tde_ctx* ctx, const float* x, int64_t n, int bits, float inv_step,
                 int8_t* q, tde_qstat* stat, void* ws, size_t ws_bytes, void* stream);

/* Quantizer kinds. Section 3.2 admits any monotone map with integer range
 * (non-uniform ones included) and Section 5 names better quantizers as future
 * work. Every kind keeps the uniform quantizer's scale inv_step (above) and
 * z = fl32(x * inv_step), so |z| = K + 1/2 at 3 sigma; bits = 1 is the sign
 * map for every kind. The non-uniform kinds, for bits 2 and 4, send x to
 * sign(z) times the number of cell boundaries T_1 < ... < T_K strictly below
 * |z| (NaN to 0, +-Inf to +-K), codes in [-K, K], phi(0) = 0:
 *   TDE_QUANT_MULAW  mu-law companding, mu = 255, on [-3 sigma, 3 sigma]:
 *                    T_k = 3 ((1+mu)^((k-1/2)/(K+1/2)) - 1) / mu  (sigma units)
 *   TDE_QUANT_GAUSS  Lloyd-Max quantizer of a unit Gaussian with 2K+1 levels
 *                    (boundaries midway between levels, levels the
 *                    conditional means of their cells)
 * with sigma units turned into z units by (2K+1)/6 and rounded to float32. */
#define TDE_QUANT_UNIFORM 0
#define TDE_QUANT_MULAW   1
#define TDE_QUANT_GAUSS   2
/* tde_quantize with a quantizer kind; TDE_ERR_UNSUPPORTED for a non-uniform
 * kind with bits = 8, TDE_ERR_ARG for an unknown kind. */
int tde_quantize_ex(tde_ctx* ctx, const float* x, int64_t n, int bits, int quantizer, float inv_step,
                    int8_t* q, tde_qstat* stat, void* ws, size_t ws_bytes, void* stream);
/* Writes the K boundaries T_k (z units, float32, ascending) of a non-uniform
 * kind at bits 2 or 4 into out (host, room for 7) and returns K; TDE_ERR_ARG
 * for another kind or a null out, TDE_ERR_UNSUPPORTED for other bits. */
int tde_quantizer_thresholds(int quantizer, int bits, float* out);

/* ------------------------------------------------------ correlation -- */

/* Algorithm 1, correlation step (Eq. (1) on integer sequences), exact:
 *   r[i] = sum_m u[m] v[m + tau],  tau = lag_lo + i,  i in [0, lag_hi - lag_lo],
 * with u on [0, nu) and v on [0, nv), zero elsewhere (finite-length signals,
 * Section 2.2). u and v (device, int8) hold codes with |u| <= kmax_u and
 * |v| <= kmax_v (1..127); kmax only sizes the overflow bound and selects
 * engines, values beyond it give undefined r. r (device) has lag_hi-lag_lo+1
 * elements of r_dtype.
 *  r_dtype = TDE_I32 requires max_tau overlap(tau) * kmax_u * kmax_v < 2^31
 *  (the coefficient bound of Section 3.2), else TDE_ERR_RANGE; TDE_I64 is
 *  always exact.
 *  path = TDE_PATH_MFMA multiplies codes up to 3 as FP4 (E2M1) and up to 7
 *  as FP6 (E2M3) with fp32 accumulation (integers, exact: every wave's
 *  partial sum stays below 2^24), larger ones as int8 with int32
 *  accumulation; TDE_PATH_MFMA_I8 takes int8 for every code range.
 *  path = TDE_PATH_POPC needs kmax_u = kmax_v = 1. TDE_PATH_NTT takes
 *  transforms up to 2^23 points (TDE_ERR_UNSUPPORTED beyond): the smallest
 *  power of two n with no alias on the requested lags inside the support,
 *  n > max(hi + nu - 1, nv - 1 - lo) for the clamped range [lo, hi], so
 *  nu + nv - 1 <= 2^23 for the full range. TDE_PATH_AUTO lets the tuning
 *  table choose.
 * Errors: TDE_ERR_ARG (nu, nv < 1, lag_lo > lag_hi, null pointers, kmax out
 * of range), TDE_ERR_RANGE, TDE_ERR_WS.
 * tde_xcorr_workspace_size returns 0 (and sets the last error) for a request
 * that tde_xcorr_int refuses for its sizes, code ranges, lag range (more
 * than 2^40 lags) or engine. */
size_t tde_xcorr_workspace_size(int64_t nu, int64_t nv, int kmax_u, int kmax_v,
                                int64_t lag_lo, int64_t lag_hi, int path);
/* Operand width (4, 6 or 8 bits) the matrix-core engine multiplies codes of
 * these ranges in, for path TDE_PATH_AUTO, _MFMA or _MFMA_I8 (the choice
 * above).
 * Errors: TDE_ERR_ARG (kmax out of [1, 127], another path). */
int tde_mfma_operand_bits(int kmax_u, int kmax_v, int path);
/* Lags per tile (4096 or 8192) the matrix-core engine cuts this correlation
 * into, for path TDE_PATH_AUTO, _MFMA or _MFMA_I8: the tuning table's tile
 * width for its bucket, else the built-in rule. Errors: TDE_ERR_ARG. */
int tde_mfma_tile_lags(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi, int path);
int tde_xcorr_int(tde_ctx* ctx, const int8_t* u, int64_t nu, const int8_t* v, int64_t nv,
                  int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi,
                  void* r, int r_dtype, int path, void* ws, size_t ws_bytes, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation):
 * tde_xcorr_int without a workspace argument. Its scratch is a static
 * device array of 16 MiB per device (one copy per GPU, held until the
 * process ends), whose address tde_create looks up; the call allocates
 * nothing, host or device. Same arguments, results and errors as
 * tde_xcorr_int, plus TDE_ERR_UNSUPPORTED when the correlation needs more
 * scratch than 16 MiB (tde_xcorr_workspace_size for the engine `path`
 * selects). Calls on one device share that scratch: calls whose work
 * overlaps in time on one GPU (different streams, or threads) race and
 * must be serialised by the caller. */
int tde_xcorr_int_noalloc(tde_ctx* ctx, const int8_t* u, int64_t nu, const int8_t* v, int64_t nv,
                          int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi,
                          void* r, int r_dtype, int path, void* stream);

/* Algorithm 1, argmax step: over r[0 .. lag_hi-lag_lo] (device, r_dtype), writes
 * *out (device) = {smallest tau with r = max, max, number of maximisers, 0}.
 * Errors: TDE_ERR_ARG. ws: tde_argmax_workspace_size(lag_hi-lag_lo+1). */
size_t tde_argmax_workspace_size(int64_t nlags);
int tde_argmax_lag(tde_ctx* ctx, const void* r, int r_dtype, int64_t lag_lo, int64_t lag_hi,
                   tde_peak* out, void* ws, size_t ws_bytes, void* stream);

/* Algorithm 1, tie-refinement step: if *peak (device, from tde_argmax_lag or a batch
 * call with r_out) has n_ties > 1, the real correlation (Eq. (1) on the float
 * signals x, y (device)) is evaluated at the tied lags of r (device, the
 * lags [lag_lo, lag_hi] in r_dtype) and *peak becomes {smallest lag of the
 * refined set, the same integer rmax, size of the refined set, flags |
 * TDE_FLAG_REFINED}. The refined set is the tied lags whose EXACT real
 * correlation is largest (no summation order enters): float64 sums with a
 * rigorous error bound decide where they can, exact sums of the products
 * (each product of two float32 values is an integer times 2^-298) decide the
 * rest (then TDE_FLAG_REFINE_EXACT is also set). If any tied lag's overlap
 * holds a NaN or Inf sample, the real correlations cannot be compared: the
 * peak keeps its lag and n_ties and gains TDE_FLAG_REFINE_NONFINITE only. At
 * most max_ties tied lags (the smallest ones, 2 <= max_ties <= 65536) are
 * considered; more set TDE_FLAG_REFINE_PARTIAL. A peak with n_ties <= 1 is
 * left unchanged. Errors: TDE_ERR_ARG (also for more than 2^31 - 1 lags),
 * TDE_ERR_WS, TDE_ERR_UNSUPPORTED when min(nx, ny) > 2^22.
 * ws: tde_refine_workspace_size(max_ties) bytes. */
size_t tde_refine_workspace_size(int max_ties);
int tde_refine_ties(tde_ctx* ctx, const float* x, int64_t nx, const float* y, int64_t ny, const void* r,
                    int r_dtype, int64_t lag_lo, int64_t lag_hi, tde_peak* peak, int max_ties, void* ws,
                    size_t ws_bytes, void* stream);

/* --------------------------------------------------------- streaming -- */

/* Correlation of a stream against a template, block by block (overlap-save):
 * the extension to long and streaming signals that Section 5 names as future
 * work, built from the steps of Algorithm 1 from quantization to argmax. The
 * template x (device float32, nx samples) is quantized once with bits in
 * {1,2,4,8} at inv_step_x (0: its own scale, as in tde_quantize); every stream block is
 * quantized at the one fixed scale inv_step_y (> 0; ignored for bits = 1), so
 * the stream's codes are those of the concatenation. With u the template's
 * codes and v the stream's, zero outside [0, T) for T samples pushed,
 *   r[tau] = sum_m u[m] v[m + tau]          (Eq. (1))
 * is final for tau <= T - nx. A push of n samples makes the n lags
 * [T - nx + 1, T + n - nx] final (T before the push); tde_stream_finish makes
 * the last nx - 1 lags [T - nx + 1, T - 1] final, with zeros after the end,
 * and ends the stream. Each call computes its lags exactly on the engine
 * `path` selects (as tde_xcorr_int: the template against the last nx - 1 + n
 * codes of the stream) and
 *   r_out (device, may be NULL): its lags' r, r_dtype (TDE_I32 requires
 *     nx * K^2 < 2^31, K the bits' largest code);
 *   block_peak (device, may be NULL): the argmax of its lags (smallest lag,
 *     max, count; flags 0);
 *   running_peak (device, may be NULL): the argmax over every final lag so
 *     far (ties across calls add up; the smallest lag wins).
 * Work is queued on `stream`; a stream object is used by one host thread at
 * a time and its calls must follow each other on one HIP stream. Pushes of
 * max_block samples with r_out NULL replay a plan made at creation when the
 * matrix-core engine takes such calls whole (no host work, no wait).
 * tde_stream_create allocates device memory (template codes, two history
 * buffers of nx - 1 + max(max_block, nx - 1) codes, r and engine workspace)
 * and returns TDE_ERR_ARG for null pointers, nx < 1, bad bits, a non-finite
 * or negative scale, inv_step_y = 0 with bits > 1, max_block < 1, a path
 * that is not AUTO/MFMA/MFMA_I8/POPC/NTT or does not fit the codes (POPC
 * needs bits = 1), TDE_ERR_UNSUPPORTED when the NTT engine cannot take the
 * largest call. tde_stream_push returns TDE_ERR_ARG for n < 1,
 * n > max_block, a null y, a bad r_dtype or a finished stream, TDE_ERR_RANGE
 * for TDE_I32 beyond the bound. The finishing call of a template of one
 * sample has no lags: it writes no r and leaves block_peak unchanged. */
typedef struct tde_stream tde_stream;
int tde_stream_create(tde_ctx* ctx, const float* x, int64_t nx, int bits, float inv_step_x, float inv_step_y,
                      int64_t max_block, int path, tde_stream** out, void* stream);
int tde_stream_push(tde_stream* st, const float* y, int64_t n, void* r_out, int r_dtype, tde_peak* block_peak,
                    tde_peak* running_peak, void* stream);
int tde_stream_finish(tde_stream* st, void* r_out, int r_dtype, tde_peak* block_peak, tde_peak* running_peak,
                      void* stream);
/* samples pushed so far (-1 for a null stream) */
int64_t tde_stream_position(const tde_stream* st);
/* waits for the device, then frees the stream (NULL is ignored) */
void tde_stream_destroy(tde_stream* st);

/* ------------------------------------------------------------ batch -- */

/* One pair of the batch. x, y: device float32 signals of nx, ny samples.
 * Lags [lag_lo, lag_hi]; bits in {1,2,4,8}; inv_step_* <= 0 selects the
 * automatic scale of tde_quantize. r_out (device, may be NULL): when set,
 * receives r over the lag range in r_dtype. */
typedef struct {
    const float* x;
    const float* y;
    int64_t nx, ny;
    int64_t lag_lo, lag_hi;
    int32_t bits;
    float   inv_step_x, inv_step_y;
    int32_t r_dtype;
    void*   r_out;
} tde_pair;

#define TDE_MODE_FULL    0
#define TDE_MODE_LEARNED 1

typedef struct tde_model tde_model;

typedef struct {
    int32_t mode;            /* TDE_MODE_FULL or TDE_MODE_LEARNED */
    int32_t path;            /* TDE_PATH_* forced for every pair, or AUTO */
    int32_t use_graph;       /* see below */
    int32_t topk;            /* learned mode: windows (bins) per pair, 1..16 */
    const tde_model* model;  /* learned mode: the proposer */
    float margin;            /* learned mode: full-range fallback below this logit margin
                                (-inf: never, +inf: always; NaN is rejected) */
    int32_t quantizer;       /* TDE_QUANT_* for every pair (non-uniform kinds: bits 1, 2, 4
                                only, else TDE_ERR_UNSUPPORTED) */
} tde_opts;

/* TDE_MODE_LEARNED: the model scores the nbins lag bins of every pair (see
 * the learned model section); if the margin logit_(1) - logit_(topk+1) is at
 * least opts->margin, the exact correlation runs only on the topk best bins
 * and out[i] is the argmax (smallest lag, max, count) of r restricted to
 * their union; otherwise the pair falls back to the full lag range and
 * out[i].flags carries TDE_FLAG_FALLBACK. Requirements: every pair has
 * nx = ny = 16 ld, bits in {2,4,8}, lag_lo = -(nbins/2) 256 and lag_hi =
 * (nbins/2) 256 - 1 (the union of the bins), r_out NULL; path AUTO, MFMA or
 * MFMA_I8 (the engine of the fallback). */

/* use_graph = 1: the first call with a given signature (the bytes of the
 * pairs array, opts, ws, ws_bytes and out) waits for the caller's stream,
 * writes its descriptors into the workspace and captures its kernels into a
 * HIP graph; later calls with the same signature only launch that graph on
 * the caller's stream (new sample values in the same device buffers are
 * picked up). The workspace then keeps state between calls: the caller must
 * not write to it while such calls continue. Any other call of the same
 * context whose workspace overlaps it drops the cached graph. Stage timing
 * is not recorded for graph launches. */

/* Algorithm 1 up to its argmax step for every pair of pairs_host[0..npairs) (host array):
 * quantize x and y, correlate exactly, and write out[i] (device) for pair i.
 * Pairs may differ in length, lag range and bits. Errors: TDE_ERR_ARG for an
 * invalid pair (the message names it), TDE_ERR_RANGE if a requested int32 r
 * cannot hold the exact values, TDE_ERR_WS. */
size_t tde_estimate_workspace_size(const tde_pair* pairs_host, int64_t npairs, const tde_opts* opts);
int tde_estimate_batch(tde_ctx* ctx, const tde_pair* pairs_host, int64_t npairs,
                       const tde_opts* opts, tde_peak* out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------ learned model -- */

/* Learned lag-window proposer. Not part of the paper: it only chooses where
 * Algorithm 1's exact correlation step is evaluated, and the full lag
 * range remains the fallback, so results stay exact. Architecture (fixed):
 *   input   xd[t] = bf16(mean of x[16t .. 16t+15] / sigma), t < ld, with
 *           sigma = sqrt(S/n) of the quantizer scale (Section on the scale in
 *           tde_quantize); both signals of a pair go through the same encoder
 *   encoder 4 x [conv1d kernel 9, zero padding 4, 32 channels, bias, ReLU,
 *           average pooling of 2] -> 32 x F features, F = ld / 16
 *   head    logits[k] = alpha sum_t sum_c Fx[c][t] Fy[c][t + k - nbins/2],
 *           k < nbins: bin k covers the lags [(k - nbins/2) 256,
 *           (k - nbins/2 + 1) 256) of the raw signals (one feature step is
 *           256 samples)
 * Parameters (float32, in this order): for each layer l, W_l[32][cin][9]
 * (cin = 1 for l = 0, else 32) then b_l[32]; then alpha. Kernels use
 * bf16-rounded copies of the weights and bf16 activations with float32
 * accumulation (alpha stays float32). Training: softmax cross-entropy against a bin label, Adam
 * (beta 0.9 / 0.999, eps 1e-8) on float32 masters.
 *
 * These are support calls, not hot calls: they may allocate device memory
 * (model parameters, training buffers sized for the largest batch seen) and
 * synchronize. xdec arrays hold bf16 bit patterns, [B][2][ld] (x then y). */
/* ld: multiple of 256 in [256, 2^20]; nbins: multiple of 64, at most 2 ld/16
 * and 1024. Weights start He-normal from `seed`, biases 0, alpha 1/(32 F). */
int tde_model_create(tde_ctx* ctx, int ld, int nbins, uint64_t seed, tde_model** out);
void tde_model_destroy(tde_model* model);
int64_t tde_model_num_params(const tde_model* model);
/* Host copies of the float32 parameters (n = tde_model_num_params). Setting
 * them also resets the Adam state. */
int tde_model_get_params(tde_model* model, float* host, int64_t n);
int tde_model_set_params(tde_model* model, const float* host, int64_t n);
/* Gradient of the mean loss from the last tde_train_step (host copy). */
int tde_model_gradients(tde_model* model, float* host, int64_t n);
/* Checkpoint file: magic "TDE2", ld, nbins, count, Adam step (int32), then
 * the float32 parameters and Adam's first and second moments, so a training
 * run resumed from it continues bit for bit. Load also takes the older
 * parameters-only files (magic "TDE1"; the Adam state then restarts) and
 * fails with TDE_ERR_IO for a file of another shape, a short or over-long
 * file, or invalid moments. */
int tde_model_save(tde_model* model, const char* path);
int tde_model_load(tde_model* model, const char* path);

/* Decimated, normalised inputs of npairs pairs (pairs_host as for
 * tde_estimate_batch; every pair has nx = ny = 16 ld and bits in {2,4,8},
 * whose automatic scale gives sigma) into xdec [npairs][2][ld] (device). ws:
 * tde_model_prepare_workspace_size bytes. */
size_t tde_model_prepare_workspace_size(const tde_pair* pairs_host, int64_t npairs);
int tde_model_prepare(tde_ctx* ctx, const tde_model* model, const tde_pair* pairs_host, int64_t npairs,
                      uint16_t* xdec, void* ws, size_t ws_bytes, void* stream);

/* logits [B][nbins] (device) of B input pairs; with top and margin (device,
 * may both be NULL) also the topk best bins per pair (descending logit, ties
 * to the smaller bin; 1 <= topk <= 16) and margin = logit_(1) - logit_(topk+1). */
int tde_model_forward(tde_ctx* ctx, tde_model* model, const uint16_t* xdec, int64_t B, float* logits, int topk,
                      int32_t* top, float* margin, void* stream);
/* One Adam step on the mean softmax cross-entropy of B pairs against labels
 * (device int32 bins). loss_out (host, may be NULL) receives the mean loss
 * (the call then waits for the stream). */
int tde_train_step(tde_ctx* ctx, tde_model* model, const uint16_t* xdec, const int32_t* labels, int64_t B, float lr,
                   float* loss_out, void* stream);

/* ------------------------------------------------------------ tuning -- */

/* TDE_PATH_AUTO picks the engine of each correlation from a tuning table
 * shared by every context of the process, keyed on the size bucket
 * round(log2(max(nu, nv))) in [10, 23], the requested fraction of the full
 * linear lag range (<= 1/16, <= 1/2, more) and the code class (Ku Kv = 1,
 * <= 49, larger). The table also holds, per bucket, the matrix-core
 * engine's tile width (4 or 8 accumulator blocks of 1024 lags), used by
 * every matrix-core correlation of the bucket whatever its path. Without a
 * table a built-in cost model picks the engine and a rule the tile width.
 * All engines and tiles give identical results; only speed differs.
 * Workspace sizes assume the table in place at that moment: install or
 * change the table before sizing workspaces (a call with a too-small
 * workspace returns TDE_ERR_WS). */

/* Measure every applicable engine (the matrix-core engine at both tile
 * widths) for sizes 2^10 .. 2^max_log_n (max_log_n in [10, 22]) and all
 * buckets, and install the fastest engine and tile width per bucket; larger
 * sizes take the largest measured bucket. Each bucket is timed as the batch
 * call runs it: a batch of identical synthetic pairs (b = 1, 4 or 8 for the
 * three code classes) large enough to fill the device, scored per pair. Not
 * a hot call: it allocates its own device buffers and synchronizes `stream`. */
int tde_tune(tde_ctx* ctx, int max_log_n, void* stream);
/* The engine (TDE_PATH_MFMA, _POPC or _NTT) that TDE_PATH_AUTO takes for this
 * correlation, or TDE_ERR_ARG. */
int tde_tune_query(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi);
/* Text file: a line "tde-tune 2", then lines "code_class lag_class log2n
 * engine tile_blocks" (tile_blocks 4, 8, or 0 for the rule); files of
 * version 1 (no tile column) still load. Save fails with TDE_ERR_ARG when no
 * table is installed; load replaces the table (TDE_ERR_IO for an unreadable
 * or malformed file, which leaves the table unchanged); reset returns to the
 * cost model and the tile rule. */
int tde_tune_save(const char* path);
int tde_tune_load(const char* path);
int tde_tune_reset(void);

/* ------------------------------------------------------ measurement -- */

/* Stage timing of tde_estimate_batch, for benchmarks. While enabled, each
 * call records HIP events on the caller's stream around its stages:
 *   0 quantize (scale + codes), 1 correlation engine (in learned mode also
 *   the proposer), 2 argmax, 3 whole call, 4 proposer (learned mode: CNN
 *   forward and top-k, a part of stage 1), 5 windowed exact correlation
 *   (learned mode, a part of stage 1), 6 the matrix-core engine's launch
 *   (a part of stage 1; in learned mode the full-range fallback).
 * tde_timing_read waits for the recorded events, writes the summed
 * milliseconds and the number of timed calls per stage to ms[TDE_STAGES]
 * and count[TDE_STAGES] (host arrays), and clears the record. Enabling
 * allocates events; the estimate call itself still allocates no device
 * memory. */
#define TDE_STAGES 7
int tde_timing_enable(tde_ctx* ctx, int on);
int tde_timing_read(tde_ctx* ctx, double* ms, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* TDE_H */
