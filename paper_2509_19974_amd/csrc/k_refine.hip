// Algorithm 1, tie-refinement step: when the integer correlation has several maximising
// lags (Remark 1), the real-valued correlation (Eq. (1) on the unquantized
// signals) decides among them. The products x[m] y[m + tau] are exact in
// float64; they are added over a fixed binary tree (ascending m, zero-padded
// to a power of two, adjacent pairs level by level), so the choice between
// tied lags is reproducible bit for bit.
//
//   k_tie_collect   one workgroup: the tied lags of r (r == rmax), in
//                   increasing order, at most max_ties of them
//   k_tie_dot       one workgroup per collected lag: the float64 tree sum
//   k_tie_final     the refined set: maximum value, smallest lag, its size
#include "tde_internal.h"

namespace tde {

namespace {

__device__ __forceinline__ int64_t r_at(const void* r, int dtype, int64_t i) {
    return dtype == TDE_I32 ? (int64_t) static_cast<const int32_t*>(r)[i] : static_cast<const int64_t*>(r)[i];
}

}  // namespace

__global__ void __launch_bounds__(256) k_tie_collect(const void* r, int dtype, int64_t L, const tde_peak* peak,
                                                     int64_t lag_lo, int max_ties, int64_t* lags, int* count) {
    __shared__ int s_base;
    __shared__ int s_wave[4];
    const int64_t rmax = peak->rmax;
    const bool todo = peak->n_ties > 1;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t b = 0; todo && b < L; b += 256) {
        const int64_t i = b + threadIdx.x;
        const bool hit = i < L && r_at(r, dtype, i) == rmax;
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
    if (threadIdx.x == 0) *count = todo ? s_base : 0;
}

// grid max_ties; workgroup k sums lag lags[k] (if k < count).
__global__ void __launch_bounds__(256) k_tie_dot(const float* x, int64_t nx, const float* y, int64_t ny,
                                                 const int64_t* lags, const int* count, int max_ties, double* vals) {
    const int k = blockIdx.x;
    const int n = *count < max_ties ? *count : max_ties;
    if (k >= n) return;
    const int64_t tau = lags[k];
    const int64_t lo = tau < 0 ? -tau : 0;
    const int64_t hi = nx < ny - tau ? nx : ny - tau;
    const int64_t M = hi > lo ? hi - lo : 0;
    const int64_t nblk = (M + 1023) / 1024;
    __shared__ double nodes[4096];
    __shared__ double wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // level-10 nodes (1024 products each), one block at a time
    int64_t nn = 1;
    while (nn < nblk) nn *= 2;
    // more than 4096 level-10 nodes (M > 2^22) is refused by the host
    for (int64_t blk = 0; blk < nn; ++blk) {
        double a = 0.0;
        if (blk < nblk) {
            double p[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t idx = blk * 1024 + 4 * threadIdx.x + e;
                p[e] = idx < M ? (double)x[lo + idx] * (double)y[lo + idx + tau] : 0.0;
            }
            a = (p[0] + p[1]) + (p[2] + p[3]);
#pragma unroll
            for (int h = 1; h < 64; h <<= 1) a = a + __shfl_xor(a, h, 64);
        }
        if (lane == 0) wsum[w] = a;
        __syncthreads();
        if (threadIdx.x == 0) nodes[blk] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        __syncthreads();
    }
    // levels above: read a whole level, then write it (levels span waves)
    for (int64_t h = nn / 2; h >= 1; h /= 2) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t i = threadIdx.x + 256 * q;
            if (i < h) v[q] = nodes[2 * i] + nodes[2 * i + 1];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t i = threadIdx.x + 256 * q;
            if (i < h) nodes[i] = v[q];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) vals[k] = nodes[0];
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

int launch_refine(const float* x, int64_t nx, const float* y, int64_t ny, const void* r, int dtype, int64_t lag_lo,
                  int64_t L, tde_peak* peak, int max_ties, int64_t* lags, double* vals, int* count, hipStream_t s) {
    hipLaunchKernelGGL(k_tie_collect, dim3(1), dim3(256), 0, s, r, dtype, L, peak, lag_lo, max_ties, lags, count);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_dot, dim3(max_ties), dim3(256), 0, s, x, nx, y, ny, lags, count, max_ties, vals);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_tie_final, dim3(1), dim3(64), 0, s, peak, lags, vals, count, max_ties);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
