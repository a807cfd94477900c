// Algorithm 1, tie-refinement step: when the integer correlation has several maximising
// lags (Remark 1), the real-valued correlation (Eq. (1) on the unquantized
// signals) decides among them. The refined set is the tied lags whose exact
// real correlation is largest; the exact values have no summation order.
//
//   k_tie_count     one workgroup per chunk of r: its hits (r == rmax)
//   k_tie_collect   one workgroup per chunk: its tied lags, in increasing
//                   order after those of the chunks before it, the first
//                   max_ties overall, and the total count
//   k_tie_dot       one workgroup per collected lag: the float64 tree sum of
//                   the products x[m] y[m + tau] (each exact in float64) and
//                   of their magnitudes, which bounds the tree sum's error
//   k_tie_select    the lags whose interval [sum - bound, sum + bound] can
//                   still hold the maximum; a single one is the refined set
//   k_tie_exact     the exact sums of the remaining candidates (integer
//                   digits, no rounding)
//   k_tie_final     the refined set among them: exact maximum, smallest lag,
//                   its size
// A tied lag whose overlap holds a NaN or Inf sample has no real correlation
// to compare: the peak is then left unrefined and flagged.
#include "exact_sum.h"
#include "tde_internal.h"

namespace tde {

namespace {

__device__ __forceinline__ int64_t r_at(const void* r, int dtype, int64_t i) {
    return dtype == TDE_I32 ? (int64_t) static_cast<const int32_t*>(r)[i] : static_cast<const int64_t*>(r)[i];
}

}  // namespace

// Collect, pass 1: the hits (r == rmax) of each chunk of `chunk` entries.
__global__ void __launch_bounds__(256) k_tie_count(const void* r, int dtype, int64_t L, int64_t chunk,
                                                   const tde_peak* peak, int* hits) {
    __shared__ int s_wave[4];
    const int64_t rmax = peak->rmax;
    const bool todo = peak->n_ties > 1;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = c0 + chunk < L ? c0 + chunk : L;
    int h = 0;
    if (todo) {
#pragma unroll 8
        for (int64_t i = c0 + threadIdx.x; i < c1; i += 256) h += r_at(r, dtype, i) == rmax ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = h;
    __syncthreads();
    if (threadIdx.x == 0) hits[blockIdx.x] = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
}

// Collect, pass 2: each chunk writes its tied lags in increasing order from
// the offset that the hits of the chunks before it give, keeping the first
// max_ties overall; the last chunk writes the total count (0 when the peak
// has a single maximiser).
__global__ void __launch_bounds__(256) k_tie_collect(const void* r, int dtype, int64_t L, int64_t chunk,
                                                     const tde_peak* peak, int64_t lag_lo, int max_ties,
                                                     const int* hits, int64_t* lags, int* count) {
    __shared__ int s_wave[4];
    __shared__ int s_base;
    const int64_t rmax = peak->rmax;
    const bool todo = peak->n_ties > 1;
    const int g = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int pre = 0;
    for (int j = threadIdx.x; j < g; j += 256) pre += hits[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if (lane == 0) s_wave[w] = pre;
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        if (g == (int)gridDim.x - 1) *count = todo ? s_base + hits[g] : 0;
    }
    __syncthreads();
    // the same decision in every thread of the workgroup
    if (!todo || s_base >= max_ties || hits[g] == 0) return;
    const int64_t c0 = (int64_t)g * chunk;
    const int64_t c1 = c0 + chunk < L ? c0 + chunk : L;
    for (int64_t b = c0; b < c1; b += 256) {
        const int64_t i = b + threadIdx.x;
        const bool hit = i < c1 && r_at(r, dtype, i) == rmax;
        const unsigned long long m = __ballot(hit);
        if (lane == 0) s_wave[w] = __popcll(m);
        __syncthreads();
        int off = s_base;
        for (int k = 0; k < w; ++k) off += s_wave[k];
        off += __popcll(m & ((1ull << lane) - 1ull));
        if (hit && off < max_ties) lags[off] = lag_lo + i;
        __syncthreads();
        if (threadIdx.x == 0) s_base += s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        __syncthreads();
        if (s_base >= max_ties) break;
    }
}

// Workgroup g sums the lags lags[k], k = g, g + grid, ... below
// min(count, max_ties). Wave w takes the 1024-product blocks w, w + 16, ...;
// in a block, lane l holds products 256 s + 4 l .. 256 s + 4 l + 3
// (s = 0..3) and adds them ((p0 + p1) + (p2 + p3)), the 64 lanes then give
// the 256-product subtree S_s, and ((S0 + S1) + (S2 + S3)) is the block's
// node; the nodes are added as a power-of-two tree. The same tree adds the
// magnitudes |p|, so vals[k] = the sum and errs[k] = 2^-45 times the sum of
// magnitudes bounds |vals[k] - exact| (a tree of height at most 64). Any
// NaN or Inf sample in the overlap makes errs[k] non-finite (finite
// products stay below 2^256 and their sums below 2^278, so nothing else
// overflows). All 32 loads of a block are issued before any product is formed.
constexpr int kDotThreads = 1024;
__global__ void __launch_bounds__(kDotThreads) k_tie_dot(const float* x, int64_t nx, const float* y, int64_t ny,
                                                         const int64_t* lags, const int* count, int max_ties,
                                                         double* vals, double* errs) {
    const int n = *count < max_ties ? *count : max_ties;
    __shared__ double nodes[4096];
    __shared__ double anodes[4096];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const int64_t tau = lags[k];
        const int64_t lo = tau < 0 ? -tau : 0;
        const int64_t hi = nx < ny - tau ? nx : ny - tau;
        const int64_t M = hi > lo ? hi - lo : 0;
        const int64_t nblk = (M + 1023) / 1024;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        constexpr int kWaves = kDotThreads / 64;
        // padded to a power of two; more than 4096 nodes (M > 2^22) is
        // refused by the host
        int64_t nn = 1;
        while (nn < nblk) nn *= 2;
        const float* xs = x + lo;
        const float* ys = y + lo + tau;
        for (int64_t blk = w; blk < nn; blk += kWaves) {
            double node = 0.0, anode = 0.0;
            if (blk < nblk) {
                float xv[16], yv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int64_t idx = blk * 1024 + 256 * (q >> 2) + 4 * lane + (q & 3);
                    xv[q] = idx < M ? xs[idx] : 0.f;
                    yv[q] = idx < M ? ys[idx] : 0.f;
                }
                double S[4], A[4];
#pragma unroll
                for (int sb = 0; sb < 4; ++sb) {
                    double p[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) p[e] = (double)xv[4 * sb + e] * (double)yv[4 * sb + e];
                    double a = (p[0] + p[1]) + (p[2] + p[3]);
                    double b = (__builtin_fabs(p[0]) + __builtin_fabs(p[1])) +
                               (__builtin_fabs(p[2]) + __builtin_fabs(p[3]));
#pragma unroll
                    for (int h = 1; h < 64; h <<= 1) {
                        a = a + __shfl_xor(a, h, 64);
                        b = b + __shfl_xor(b, h, 64);
                    }
                    S[sb] = a;
                    A[sb] = b;
                }
                node = (S[0] + S[1]) + (S[2] + S[3]);
                anode = (A[0] + A[1]) + (A[2] + A[3]);
            }
            if (lane == 0) {
                nodes[blk] = node;
                anodes[blk] = anode;
            }
        }
        __syncthreads();
        // levels above: read a whole level, then write it (levels span waves)
        constexpr int kQ = 2048 / kDotThreads;
        for (int64_t h = nn / 2; h >= 1; h /= 2) {
            double v[kQ], av[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int64_t i = threadIdx.x + kDotThreads * q;
                if (i < h) {
                    v[q] = nodes[2 * i] + nodes[2 * i + 1];
                    av[q] = anodes[2 * i] + anodes[2 * i + 1];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int64_t i = threadIdx.x + kDotThreads * q;
                if (i < h) {
                    nodes[i] = v[q];
                    anodes[i] = av[q];
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            vals[k] = nodes[0];
            errs[k] = anodes[0] * kTreeRelErr;
        }
        __syncthreads();      // nodes are rewritten for the next lag
    }
}

namespace {
__device__ __forceinline__ void set_peak(tde_peak* peak, int64_t lag, int n_ties, int flags, bool keep) {
    tde_peak pk = *peak;
    if (!keep) {
        pk.lag = lag;
        pk.n_ties = n_ties;
    }
    pk.flags |= flags;
    *peak = pk;
}
}  // namespace

// One workgroup. With every tied lag's bound finite: lo_max = max (val -
// err) is at most the exact maximum, so only lags with val + err >= lo_max
// can attain it. A single such lag is the refined set (every other exact
// value lies strictly below it); several go to the exact sums. A non-finite
// bound (NaN or Inf in an overlap) leaves the peak unrefined.
__global__ void __launch_bounds__(256) k_tie_select(tde_peak* peak, const int64_t* lags, const double* vals,
                                                    const double* errs, const int* count, int max_ties, int* cand,
                                                    int* ncand) {
    __shared__ double s_lo[4];
    __shared__ int s_bad[4];
    __shared__ int s_n;
    const int c = *count;
    if (threadIdx.x == 0) s_n = 0;
    if (c <= 1) {
        if (threadIdx.x == 0) *ncand = 0;
        return;
    }
    const int n = c < max_ties ? c : max_ties;
    const int partial = c > max_ties ? TDE_FLAG_REFINE_PARTIAL : 0;
    double lo = -INFINITY;
    int bad = 0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const double e = errs[k];
        if (!__builtin_isfinite(e)) bad = 1;
        else lo = fmax(lo, vals[k] - e);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmax(lo, __shfl_xor(lo, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_bad[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    const double lo_max = fmax(fmax(s_lo[0], s_lo[1]), fmax(s_lo[2], s_lo[3]));
    if (s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]) {
        if (threadIdx.x == 0) {
            *ncand = 0;
            set_peak(peak, 0, 0, TDE_FLAG_REFINE_NONFINITE | partial, true);
        }
        return;
    }
    for (int k = threadIdx.x; k < n; k += 256) {
        if (vals[k] + errs[k] >= lo_max) {
            const int at = atomicAdd(&s_n, 1);
            cand[at] = k;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_n == 1) {
            set_peak(peak, lags[cand[0]], 1, TDE_FLAG_REFINED | partial, false);
            *ncand = 0;
        } else {
            *ncand = s_n;
        }
    }
}

// Exact real correlation of each candidate lag: the products as integer
// digits (exact_sum.h) added into a column of kExactLimbs int64 limbs per
// thread (at most 2^14 terms each, so no limb leaves int64), each column
// normalised, the columns added per limb (below 2^40 each), and the sum
// normalised again: limbs[c][0 .. kExactLimbs) holds candidate c's value.
constexpr int kExactThreads = 256;
__global__ void __launch_bounds__(kExactThreads) k_tie_exact(const float* x, int64_t nx, const float* y, int64_t ny,
                                                             const int64_t* lags, const int* cand, const int* ncand,
                                                             int64_t* limbs) {
    __shared__ int64_t acc[kExactLimbs][kExactThreads];
    __shared__ int64_t tot[kExactLimbs];
    const int nc = *ncand;
    const int t = threadIdx.x;
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        const int64_t tau = lags[cand[c]];
        const int64_t lo = tau < 0 ? -tau : 0;
        const int64_t hi = nx < ny - tau ? nx : ny - tau;
        for (int i = 0; i < kExactLimbs; ++i) acc[i][t] = 0;
        for (int64_t m = lo + t; m < hi; m += kExactThreads) {
            const ExactTerm p = exact_term(x[m], y[m + tau]);
            if (p.mag == 0) continue;
            int li;
            uint32_t d0, d1, d2;
            exact_digits(p, li, d0, d1, d2);
            const int64_t sg = p.neg ? -1 : 1;
            acc[li][t] += sg * (int64_t)d0;
            acc[li + 1][t] += sg * (int64_t)d1;
            acc[li + 2][t] += sg * (int64_t)d2;
        }
        // normalise the thread's own column
        int64_t carry = 0;
        for (int i = 0; i < kExactLimbs - 1; ++i) {
            const int64_t v = acc[i][t] + carry;
            carry = v >> 32;
            acc[i][t] = v - carry * ((int64_t)1 << 32);
        }
        acc[kExactLimbs - 1][t] += carry;
        __syncthreads();
        // wave w adds limbs w, w + 4, ... over the 256 columns
        const int lane = t & 63, w = t >> 6;
        for (int i = w; i < kExactLimbs; i += kExactThreads / 64) {
            int64_t s = acc[i][lane] + acc[i][lane + 64] + acc[i][lane + 128] + acc[i][lane + 192];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) tot[i] = s;
        }
        __syncthreads();
        if (t == 0) {
            int64_t v[kExactLimbs];
            for (int i = 0; i < kExactLimbs; ++i) v[i] = tot[i];
            exact_normalize(v);
            for (int i = 0; i < kExactLimbs; ++i) limbs[(int64_t)c * kExactLimbs + i] = v[i];
        }
        __syncthreads();      // acc and tot are rewritten for the next candidate
    }
}

// One wave: the exact maximum over the candidates, its smallest lag and how
// many candidates attain it.
__global__ void __launch_bounds__(64) k_tie_final(tde_peak* peak, const int64_t* lags, const int* cand,
                                                  const int* ncand, const int* count, int max_ties,
                                                  const int64_t* limbs) {
    const int nc = *ncand;
    if (nc <= 1) return;
    int best = -1;
    int64_t bl = INT64_MAX;
    int cnt = 0;
    for (int c = threadIdx.x; c < nc; c += 64) {
        const int64_t lag = lags[cand[c]];
        const int o = best < 0 ? 1 : exact_compare(limbs + (int64_t)c * kExactLimbs, limbs + (int64_t)best * kExactLimbs);
        if (o > 0) {
            best = c;
            bl = lag;
            cnt = 1;
        } else if (o == 0) {
            bl = lag < bl ? lag : bl;
            cnt += 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int ob = __shfl_xor(best, o, 64);
        const int64_t ol = __shfl_xor(bl, o, 64);
        const int oc = __shfl_xor(cnt, o, 64);
        int cmp;
        if (ob < 0) cmp = -1;
        else if (best < 0) cmp = 1;
        else cmp = exact_compare(limbs + (int64_t)ob * kExactLimbs, limbs + (int64_t)best * kExactLimbs);
        if (cmp > 0) {
            best = ob;
            bl = ol;
            cnt = oc;
        } else if (cmp == 0 && ob >= 0) {
            bl = ol < bl ? ol : bl;
            cnt += oc;
        }
    }
    if (threadIdx.x == 0) {
        const int partial = *count > max_ties ? TDE_FLAG_REFINE_PARTIAL : 0;
        set_peak(peak, bl, cnt, TDE_FLAG_REFINED | TDE_FLAG_REFINE_EXACT | partial, false);
    }
}

int64_t refine_chunk(int64_t L) {
    const int64_t c = round_up(ceil_div(L, kRefineMaxChunks), 256);
    return c < 1024 ? 1024 : c;
}

int launch_refine(const float* x, int64_t nx, const float* y, int64_t ny, const void* r, int dtype, int64_t lag_lo,
                  int64_t L, tde_peak* peak, int max_ties, const RefineWs& w, hipStream_t s) {
    const int64_t chunk = refine_chunk(L);
    const int nch = (int)ceil_div(L, chunk);     // at most kRefineMaxChunks
    hipLaunchKernelGGL(k_tie_count, dim3(nch), dim3(256), 0, s, r, dtype, L, chunk, peak, w.hits);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_collect, dim3(nch), dim3(256), 0, s, r, dtype, L, chunk, peak, lag_lo, max_ties, w.hits,
                       w.lags, w.count);
    TDE_HIP_CHECK(hipGetLastError());
    // one 16-wave workgroup per CU covers the chip; more tied lags loop
    const int g = max_ties < 256 ? max_ties : 256;
    hipLaunchKernelGGL(k_tie_dot, dim3(g), dim3(kDotThreads), 0, s, x, nx, y, ny, w.lags, w.count, max_ties, w.vals,
                       w.errs);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_select, dim3(1), dim3(256), 0, s, peak, w.lags, w.vals, w.errs, w.count, max_ties, w.cand,
                       w.ncand);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_exact, dim3(g), dim3(kExactThreads), 0, s, x, nx, y, ny, w.lags, w.cand, w.ncand,
                       w.limbs);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_final, dim3(1), dim3(64), 0, s, peak, w.lags, w.cand, w.ncand, w.count, max_ties,
                       w.limbs);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
