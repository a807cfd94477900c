// Algorithm 1, tie-refinement step: when the integer correlation has several maximising
// lags (Remark 1), the real-valued correlation (Eq. (1) on the unquantized
// signals) decides among them. The products x[m] y[m + tau] are exact in
// float64; they are added over a fixed binary tree (ascending m, zero-padded
// to a power of two, adjacent pairs level by level), so the choice between
// tied lags is reproducible bit for bit.
//
//   k_tie_count     one workgroup per chunk of r: its hits (r == rmax)
//   k_tie_collect   one workgroup per chunk: its tied lags, in increasing
//                   order after those of the chunks before it, the first
//                   max_ties overall, and the total count
//   k_tie_dot       one workgroup per collected lag: the float64 tree sum
//   k_tie_final     the refined set: maximum value, smallest lag, its size
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
// min(count, max_ties). Wave w takes
// the 1024-product blocks w, w + 16, ...; in a block, lane l holds products
// 256 s + 4 l .. 256 s + 4 l + 3 (s = 0..3) and adds them ((p0 + p1) +
// (p2 + p3)), the 64 lanes then give the 256-product subtree S_s, and
// ((S0 + S1) + (S2 + S3)) is the block's level-10 node of the fixed tree.
// All 32 loads of a block are issued before any product is formed.
constexpr int kDotThreads = 1024;
__global__ void __launch_bounds__(kDotThreads) k_tie_dot(const float* x, int64_t nx, const float* y, int64_t ny,
                                                         const int64_t* lags, const int* count, int max_ties,
                                                         double* vals) {
    const int n = *count < max_ties ? *count : max_ties;
    __shared__ double nodes[4096];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const int64_t tau = lags[k];
        const int64_t lo = tau < 0 ? -tau : 0;
        const int64_t hi = nx < ny - tau ? nx : ny - tau;
        const int64_t M = hi > lo ? hi - lo : 0;
        const int64_t nblk = (M + 1023) / 1024;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        constexpr int kWaves = kDotThreads / 64;
        // padded to a power of two; more than 4096 level-10 nodes (M > 2^22) is
        // refused by the host
        int64_t nn = 1;
        while (nn < nblk) nn *= 2;
        const float* xs = x + lo;
        const float* ys = y + lo + tau;
        for (int64_t blk = w; blk < nn; blk += kWaves) {
            double node = 0.0;
            if (blk < nblk) {
                float xv[16], yv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int64_t idx = blk * 1024 + 256 * (q >> 2) + 4 * lane + (q & 3);
                    xv[q] = idx < M ? xs[idx] : 0.f;
                    yv[q] = idx < M ? ys[idx] : 0.f;
                }
                double S[4];
#pragma unroll
                for (int sb = 0; sb < 4; ++sb) {
                    double p[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) p[e] = (double)xv[4 * sb + e] * (double)yv[4 * sb + e];
                    double a = (p[0] + p[1]) + (p[2] + p[3]);
#pragma unroll
                    for (int h = 1; h < 64; h <<= 1) a = a + __shfl_xor(a, h, 64);
                    S[sb] = a;
                }
                node = (S[0] + S[1]) + (S[2] + S[3]);
            }
            if (lane == 0) nodes[blk] = node;
        }
        __syncthreads();
        // levels above: read a whole level, then write it (levels span waves)
        constexpr int kQ = 2048 / kDotThreads;
        for (int64_t h = nn / 2; h >= 1; h /= 2) {
            double v[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int64_t i = threadIdx.x + kDotThreads * q;
                if (i < h) v[q] = nodes[2 * i] + nodes[2 * i + 1];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int64_t i = threadIdx.x + kDotThreads * q;
                if (i < h) nodes[i] = v[q];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) vals[k] = nodes[0];
        __syncthreads();      // nodes are rewritten for the next lag
    }
}

__global__ void __launch_bounds__(64) k_tie_final(tde_peak* peak, const int64_t* lags, const double* vals,
                                                  const int* count, int max_ties) {
    const int c = *count;
    if (c <= 1) return;
    const int n = c < max_ties ? c : max_ties;
    double best = -INFINITY;
    int64_t bl = INT64_MAX;
    int cnt = 0;
    for (int k = threadIdx.x; k < n; k += 64) {
        const double v = vals[k];
        if (v > best) {
            best = v;
            bl = lags[k];
            cnt = 1;
        } else if (v == best) {
            bl = lags[k] < bl ? lags[k] : bl;
            cnt += 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int64_t ol = __shfl_xor(bl, o, 64);
        const int oc = __shfl_xor(cnt, o, 64);
        if (ob > best) {
            best = ob;
            bl = ol;
            cnt = oc;
        } else if (ob == best) {
            bl = ol < bl ? ol : bl;
            cnt += oc;
        }
    }
    if (threadIdx.x == 0) {
        tde_peak pk = *peak;
        pk.lag = bl;
        pk.n_ties = cnt;
        pk.flags |= TDE_FLAG_REFINED | (c > max_ties ? TDE_FLAG_REFINE_PARTIAL : 0);
        *peak = pk;
    }
}

int64_t refine_chunk(int64_t L) {
    const int64_t c = round_up(ceil_div(L, kRefineMaxChunks), 256);
    return c < 1024 ? 1024 : c;
}

int launch_refine(const float* x, int64_t nx, const float* y, int64_t ny, const void* r, int dtype, int64_t lag_lo,
                  int64_t L, tde_peak* peak, int max_ties, int64_t* lags, double* vals, int* count, int* hits,
                  hipStream_t s) {
    const int64_t chunk = refine_chunk(L);
    const int nch = (int)ceil_div(L, chunk);     // at most kRefineMaxChunks
    hipLaunchKernelGGL(k_tie_count, dim3(nch), dim3(256), 0, s, r, dtype, L, chunk, peak, hits);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_collect, dim3(nch), dim3(256), 0, s, r, dtype, L, chunk, peak, lag_lo, max_ties, hits,
                       lags, count);
    TDE_HIP_CHECK(hipGetLastError());
    // one 16-wave workgroup per CU covers the chip; more tied lags loop
    hipLaunchKernelGGL(k_tie_dot, dim3(max_ties < 256 ? max_ties : 256), dim3(kDotThreads), 0, s, x, nx, y, ny, lags,
                       count, max_ties, vals);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_final, dim3(1), dim3(64), 0, s, peak, lags, vals, count, max_ties);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
