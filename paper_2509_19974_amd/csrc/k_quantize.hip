// Algorithm 1, quantization step: per-signal scale and monotone integer quantization.
//
// Scale: S = sum of x^2 over the finite samples is an exact real (the
// quantizer on [-3 sigma, 3 sigma] fixes no summation order); the scale is
// sigma = sqrt(fl64(S) / n), inv_step = fl32((2K+1) / (6 sigma)) with fl64(S)
// the exact S rounded once. The kernels add the squares (each exact in
// float64) in float64 over a binary tree: pairs inside a lane, wave
// shuffles, then LDS across waves and blocks. That sum S' satisfies
// |S' - S| <= 2^-45 S (exact_sum.h), and inv_step is a non-increasing
// function of S (every operation is correctly rounded and monotone), so
// when the ends of [S'(1 - 2^-45), S'(1 + 2^-45)] give the same inv_step,
// fl64(S) does too. Otherwise the workgroup forms S exactly (integer digits)
// and rounds it once; the statistics then carry TDE_FLAG_SCALE_EXACT.
//
// Quantizer: bits = 1 is sign with sign(0) = 0 (Section 4.2), taken from the
// IEEE bits; bits in {2,4,8} is clamp(round_half_even(fl32(x * inv_step)),
// -K, K). Both are monotone non-decreasing with phi(0) = 0 (Theorem 1).
// Non-uniform maps (any monotone integer-valued map qualifies, Section 3.2)
// keep the scale and z = fl32(x * inv_step) and count the cell boundaries
// strictly below |z|: mu-law companding (mu = 255) on [-3 sigma, 3 sigma], or
// the Lloyd-Max quantizer of a unit Gaussian with 2K+1 levels, for b in {2, 4}.
//
// The three kernels are HBM-bound: 4 bytes of x are read once for the scale
// and once for the codes, 1 byte of q is written.
#include <algorithm>
#include <cmath>

#include "tde_internal.h"

namespace tde {

constexpr int kSumBlock = 1024;    // samples per block sum (a level-10 subtree)
constexpr int kSumChunk = 4096;    // block sums reduced per LDS pass in the finalize

// Signal of a global block index. bps > 0: every signal has bps blocks, so
// the index is a division. Otherwise a 64-way search per round (one load per
// lane, a ballot), so finding the signal takes ceil(log64(nsig)) rounds
// instead of a chain of dependent loads. Every wave computes it by itself.
__device__ __forceinline__ const QSig& pick_sig(const QSig* sigs, int nsig, const QSig& one, int bps, int64_t unit,
                                                int64_t& local) {
    if (sigs == nullptr) {
        local = unit;
        return one;
    }
    if (bps > 0) {
        const uint32_t i = (uint32_t)unit / (uint32_t)bps;
        local = unit - (int64_t)i * bps;
        return sigs[i];
    }
    const int lane = threadIdx.x & 63;
    int lo = 0, n = nsig;                      // invariant: sigs[lo].blk_base <= unit
    while (n > 1) {
        const int step = (n + 63) / 64;
        const int cand = lo + lane * step;
        const bool ok = lane * step < n && sigs[cand].blk_base <= unit;
        const unsigned long long m = __ballot(ok);
        const int l = 63 - __builtin_clzll(m);
        const int nlo = lo + l * step;
        n = (lo + n - nlo) < step ? (lo + n - nlo) : step;
        lo = nlo;
    }
    local = unit - sigs[lo].blk_base;
    return sigs[lo];
}

__device__ __forceinline__ uint16_t f2bf_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ double sq_or_zero(float f) {
    double a = f;
    return __builtin_isfinite(a) ? a * a : 0.0;
}

// One block per 4096 samples of a signal: four level-10 nodes of the tree
// (1024 samples each), thread t holding samples 1024 k + 4t .. 4t+3 of node k.
// With the scale fused into the quantize kernel, this kernel also zeroes the
// statistics that kernel accumulates (first block of each signal) and the
// scratch counters of a later kernel (first block).
__global__ void __launch_bounds__(256) k_sumsq_blocks(const QSig* sigs, int nsig, QSig one, int bps, int fused,
                                                      int* zero_me, int nzero) {
    const int64_t blk = blockIdx.x;
    int64_t lb;
    const QSig& s = pick_sig(sigs, nsig, one, bps, blk, lb);
    if (fused) {
        if (blk == 0 && zero_me && (int)threadIdx.x < nzero) zero_me[threadIdx.x] = 0;
        if (lb == 0 && threadIdx.x == 0 && s.stat) {
            s.stat->flags = 0;
            s.stat->n_nonfinite = 0;
            s.stat->n_zero = 0;
            s.stat->sum_q = 0;
            s.stat->sum_q2 = 0;
        }
    }
    if (s.inv_fixed > 0.f || s.bits == 1) return;
    const int64_t base = lb * kQuantBlock;
    float4 xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t m = base + 1024 * k + 4 * (int64_t)threadIdx.x;
        if (m + 4 <= s.n && ((((uintptr_t)(s.x + m)) & 15) == 0)) {
            xv[k] = *reinterpret_cast<const float4*>(s.x + m);
        } else {
            float t4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) t4[e] = (m + e < s.n) ? s.x[m + e] : 0.f;
            xv[k] = make_float4(t4[0], t4[1], t4[2], t4[3]);
        }
    }
    __shared__ double ws[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double a = (sq_or_zero(xv[k].x) + sq_or_zero(xv[k].y)) + (sq_or_zero(xv[k].z) + sq_or_zero(xv[k].w));
#pragma unroll
        for (int h = 1; h < 64; h <<= 1) {
            double o = __shfl_xor(a, h, 64);
            a = a + o;     // lanes l and l^h hold the two children; the sum is the same in both
        }
        if ((threadIdx.x & 63) == 0) ws[k][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        const int64_t node = lb * 4 + k;
        if (node * kSumBlock < s.n) s.gsum[node] = (ws[k][0] + ws[k][1]) + (ws[k][2] + ws[k][3]);
    }
}

// inv_step of a signal from its sum of squares S: fl32((2K+1) / (6 sigma)),
// sigma = sqrt(S / n); 0 when S = 0.
__device__ __forceinline__ float scale_of_sum(double S, int64_t n, int bits) {
    if (!(S > 0.0)) return 0.f;
    const int K = (1 << (bits - 1)) - 1;
    const double var = S / (double)n;
    const double sigma = __builtin_sqrt(var);
    const double v = (double)(2 * K + 1) / (6.0 * sigma);
    return (float)v;
}

// The scale from a float64 tree sum St of the squares, if St's error bound
// decides it (St = 0 only when every square is 0, so S = 0 exactly).
__device__ __forceinline__ bool scale_decided(double St, int64_t n, int bits, float& inv) {
    if (!(St > 0.0)) {
        inv = 0.f;
        return true;
    }
    const float a = scale_of_sum(St * (1.0 - kTreeRelErr), n, bits);
    const float b = scale_of_sum(St * (1.0 + kTreeRelErr), n, bits);
    inv = a;
    return a == b;
}

// The exact sum of squares of the finite samples of x[0 .. n), n < 2^32,
// rounded once to float64, by the whole workgroup (every thread calls it).
// Each square is split into base-2^32 digits (exact_sum.h) that are added
// to one LDS row of limbs with 64-bit atomics; a limb receives at most one
// digit (< 2^32) per sample, so it stays below 2^64.
__device__ double exact_sumsq_wg(const float* x, int64_t n) {
    __shared__ unsigned long long acc[kExactLimbs];
    __shared__ double res;
    for (int i = threadIdx.x; i < kExactLimbs; i += blockDim.x) acc[i] = 0ull;
    __syncthreads();
    for (int64_t m = threadIdx.x; m < n; m += blockDim.x) {
        const float f = x[m];
        if (!__builtin_isfinite(f) || f == 0.f) continue;
        int li;
        uint32_t d0, d1, d2;
        exact_digits(exact_term(f, f), li, d0, d1, d2);
        atomicAdd(&acc[li], (unsigned long long)d0);
        if (d1) atomicAdd(&acc[li + 1], (unsigned long long)d1);
        if (d2) atomicAdd(&acc[li + 2], (unsigned long long)d2);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // unsigned carries first (a limb may exceed 2^63), then the digits
        int64_t v[kExactLimbs];
        unsigned long long carry = 0ull;
        for (int i = 0; i < kExactLimbs; ++i) {
            const unsigned long long a = acc[i] + carry;   // below 2^64: a limb plus a carry below 2^32
            v[i] = (int64_t)(a & 0xffffffffull);
            carry = a >> 32;
        }
        res = exact_to_double(v);
    }
    __syncthreads();
    return res;
}

// The whole sum tree of a signal of at most kFuseMaxN samples (at most 256
// block sums) in one wave: lane l adds block sums 4l .. 4l+3 pairwise, then
// wave shuffles take the levels above. Zeros beyond the last block sum extend
// the power-of-two tree of the finalize kernel without changing its value.
constexpr int64_t kFuseMaxN = 256 * kSumBlock;
constexpr int64_t kFuseMaxBlocks = 8192;
__device__ __forceinline__ double wave_tree_sum(const double* gsum, int64_t n) {
    const int64_t len = (n + kSumBlock - 1) / kSumBlock;
    const int l = threadIdx.x & 63;
    double v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = 4 * l + e < len ? gsum[4 * l + e] : 0.0;
    double a = (v[0] + v[1]) + (v[2] + v[3]);
#pragma unroll
    for (int h = 1; h < 64; h <<= 1) a = a + __shfl_xor(a, h, 64);
    return a;
}

// One block per signal: remaining levels of the sum tree, then the scale.
// Also zeroes the statistics that the quantize kernel accumulates.
__global__ void __launch_bounds__(256) k_scale_finalize(const QSig* sigs, int nsig, QSig one, int* zero_me,
                                                        int nzero) {
    (void)nsig;                      // the grid has one workgroup per signal
    const QSig& s = sigs ? sigs[blockIdx.x] : one;
    const int t = threadIdx.x;
    // scratch counters of a later kernel of the same call start at zero
    if (blockIdx.x == 0 && zero_me && t < nzero) zero_me[t] = 0;
    float inv;
    int exact = 0;
    if (s.bits == 1) {
        inv = 0.f;
    } else if (s.inv_fixed > 0.f) {
        inv = s.inv_fixed;
    } else {
        // levels above the 1024-sample blocks: chunks of 4096 values (each
        // a complete aligned subtree) are reduced in LDS, until one is left
        int64_t len = (s.n + kSumBlock - 1) / kSumBlock;
        double* a = s.gsum;
        double* out = a + len;
        __shared__ double st[kSumChunk];
        while (len > 1) {
            const int64_t nn = (len + kSumChunk - 1) / kSumChunk;
            for (int64_t c = 0; c < nn; ++c) {
                const int64_t lo = c * kSumChunk;
                int width = 1;
                while (width < kSumChunk && width < len - lo) width *= 2;     // padded subtree width
                for (int i = t; i < width; i += 256) st[i] = (lo + i < len) ? a[lo + i] : 0.0;
                __syncthreads();
                // one level per step: every node of the level is read before
                // any is overwritten (a level can span several waves)
                for (int h = width / 2; h >= 1; h /= 2) {
                    double v[kSumChunk / 2 / 256];
#pragma unroll
                    for (int k = 0; k < kSumChunk / 2 / 256; ++k) {
                        const int i = t + 256 * k;
                        if (i < h) v[k] = st[2 * i] + st[2 * i + 1];
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < kSumChunk / 2 / 256; ++k) {
                        const int i = t + 256 * k;
                        if (i < h) st[i] = v[k];
                    }
                    __syncthreads();
                }
                if (t == 0) out[c] = st[0];
                __syncthreads();
            }
            a = out;
            out = a + nn;
            len = nn;
        }
        if (!scale_decided(a[0], s.n, s.bits, inv)) {
            inv = scale_of_sum(exact_sumsq_wg(s.x, s.n), s.n, s.bits);
            exact = TDE_FLAG_SCALE_EXACT;
        }
    }
    if (t == 0) {
        if (s.inv_out) *s.inv_out = inv;
        if (s.stat) {
            s.stat->inv_step = inv;
            s.stat->flags = exact;
            s.stat->n_nonfinite = 0;
            s.stat->n_zero = 0;
            s.stat->sum_q = 0;
            s.stat->sum_q2 = 0;
        }
    }
}

__device__ __forceinline__ int quant1(float xf, int bits, float inv, int K, int& nonfinite, const QSig& s) {
    uint32_t b = __float_as_uint(xf);
    uint32_t mag = b & 0x7fffffffu;
    bool is_nan = mag > 0x7f800000u;
    nonfinite += (mag >= 0x7f800000u) ? 1 : 0;
    if (bits == 1) {
        if (is_nan || mag == 0) return 0;
        return (b >> 31) ? -1 : 1;
    }
    if (is_nan || inv == 0.f) return 0;
    if (s.nthr > 0) {
        const float z = __fmul_rn(xf, inv);
        const float a = __builtin_fabsf(z);
        int c = 0;
#pragma unroll
        for (int k = 0; k < 7; ++k) c += (k < s.nthr && a > s.thr[k]) ? 1 : 0;
        return z < 0.f ? -c : c;
    }
    float t = __fmul_rn(xf, inv);
    float r = __builtin_rintf(t);
    r = r > (float)K ? (float)K : r;
    r = r < -(float)K ? -(float)K : r;
    return (int)r;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// 256 threads x 16 samples per block; one set of statistic atomics per block.
// fused != 0: every block takes its signal's scale from the block sums itself
// (signals of 1 .. kFuseMaxN samples), and the first block of each signal
// publishes it.
__global__ void __launch_bounds__(256) k_quantize(const QSig* sigs, int nsig, QSig one, int bps, int fused) {
    const int64_t blk = blockIdx.x;
    int64_t lb;
    // a copy: the stores below could alias the descriptor array, which
    // would make the compiler reload its fields after every store
    const QSig s = pick_sig(sigs, nsig, one, bps, blk, lb);
    float inv;
    int exact = 0;
    if (s.bits == 1) {
        inv = 0.f;
    } else if (s.inv_fixed > 0.f) {
        inv = s.inv_fixed;
    } else if (fused) {
        // every block of the signal decides alike (same tree, same bound)
        if (!scale_decided(wave_tree_sum(s.gsum, s.n), s.n, s.bits, inv)) {
            inv = scale_of_sum(exact_sumsq_wg(s.x, s.n), s.n, s.bits);
            exact = TDE_FLAG_SCALE_EXACT;
        }
    } else {
        inv = *s.inv_out;
    }
    if (fused && lb == 0 && threadIdx.x == 0) {
        if (s.inv_out) *s.inv_out = inv;
        if (s.stat) {
            s.stat->inv_step = inv;
            s.stat->flags = exact;
        }
    }
    const int K = s.bits == 1 ? 1 : (1 << (s.bits - 1)) - 1;
    const int64_t base = lb * kQuantBlock;
    int nonfinite = 0, nzero = 0;
    int sq = 0, sq2 = 0;
    // four coalesced passes: thread t takes samples base + 1024 k + 4t + e
    float4 xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t m = base + 1024 * k + 4 * (int64_t)threadIdx.x;
        if (m + 4 <= s.n && ((((uintptr_t)(s.x + m)) & 15) == 0)) {
            xv[k] = *reinterpret_cast<const float4*>(s.x + m);
        } else {
            float t4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) t4[e] = (m + e < s.n) ? s.x[m + e] : 0.f;
            xv[k] = make_float4(t4[0], t4[1], t4[2], t4[3]);
        }
    }
    if (s.dec) {
        // fused decimation: means of 16 samples = 4 neighbouring threads,
        // summed ((x0+x1)+(x2+x3)) per thread, then lanes t^1, t^2 (the
        // same order as the stand-alone decimation kernel)
        const float scale = inv * s.dec_mul;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float a = (xv[k].x + xv[k].y) + (xv[k].z + xv[k].w);
            a += __shfl_xor(a, 1, 64);
            a += __shfl_xor(a, 2, 64);
            const int64_t m = base + 1024 * k + 4 * (int64_t)threadIdx.x;
            if ((threadIdx.x & 3) == 0 && m + 16 <= s.n) s.dec[m >> 4] = f2bf_rne(a * (1.f / 16.f) * scale);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t m = base + 1024 * k + 4 * (int64_t)threadIdx.x;
        uint32_t w = 0u;
        if (m < s.n) {
            const float xs[4] = {xv[k].x, xv[k].y, xv[k].z, xv[k].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int c = quant1(xs[e], s.bits, inv, K, nonfinite, s);
                if (m + e < s.n) {
                    nzero += c == 0;
                    sq += c;
                    sq2 += c * c;
                } else {
                    c = 0;
                }
                w |= (uint32_t)(uint8_t)c << (8 * e);
            }
            if (!s.skip_q) {
                if (m + 4 <= s.n && ((((uintptr_t)(s.q + m)) & 3) == 0)) {
                    *reinterpret_cast<uint32_t*>(s.q + m) = w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (m + e < s.n) s.q[m + e] = (int8_t)(w >> (8 * e));
                }
            }
        }
        if (s.pk) {
            // packed FP4/FP6 codes: lanes 4j .. 4j+3 hold the 16 samples of
            // one unit (4 each); a lane joins its bits with its right
            // neighbour's to form the unit's dwords
            const int W = s.pk_bits;
            const uint32_t z = W == 6 ? fp_bits4<6>(fp_bytes<6>(w)) : fp_bits4<4>(fp_bytes<4>(w));
            const uint32_t nb = __shfl_down(z, 1, 64);
            const int j = threadIdx.x & 3;
            const int64_t unit = (m - 4 * j) / 16;
            if (16 * unit < s.n) {
                if (W == 6) {
                    if (j == 0) s.pk[3 * unit] = z | (nb << 24);
                    else if (j == 1) s.pk[3 * unit + 1] = (z >> 8) | (nb << 16);
                    else if (j == 2) s.pk[3 * unit + 2] = (z >> 16) | (nb << 8);
                } else if (j == 0 || j == 2) {
                    s.pk[2 * unit + (j >> 1)] = z | (nb << 16);
                }
            }
        }
    }
    if (s.stat) {
        __shared__ long long red[4][4];
        long long a = wave_sum<long long>(nonfinite);
        long long z = wave_sum<long long>(nzero);
        long long q1 = s.stat_lite ? 0 : wave_sum<long long>(sq);
        long long q2 = s.stat_lite ? 0 : wave_sum<long long>(sq2);
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[wv][0] = a; red[wv][1] = z; red[wv][2] = q1; red[wv][3] = q2;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            long long v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
            int64_t* dst = threadIdx.x == 0 ? &s.stat->n_nonfinite
                           : threadIdx.x == 1 ? &s.stat->n_zero
                           : threadIdx.x == 2 ? &s.stat->sum_q : &s.stat->sum_q2;
            if (v) atomicAdd((unsigned long long*)dst, (unsigned long long)v);
        }
    }
}

// tde_qstat::flags from the finished counts (one thread per signal).
__global__ void k_quantize_flags(const QSig* sigs, int nsig, QSig one) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsig) return;
    const QSig& s = sigs ? sigs[i] : one;
    if (!s.stat) return;
    int f = s.stat->flags & TDE_FLAG_SCALE_EXACT;
    if (s.stat->n_nonfinite) f |= TDE_FLAG_NONFINITE_X;
    if (s.stat->n_zero == s.n) f |= TDE_FLAG_ZERO_X;
    s.stat->flags = f;
}

// Cell boundaries of the non-uniform maps, in units of sigma, then of z
// (times (2K+1)/6, the uniform quantizer's scale), rounded to float32.
//   mu-law: the compressor ln(1 + mu a/3) / ln(1 + mu) of a magnitude a (in
//     sigma) cut into K + 1/2 equal cells: a_k = 3 ((1+mu)^((k-1/2)/(K+1/2)) - 1) / mu.
//   Lloyd-Max, unit Gaussian, levels 0 and +-y_k: boundaries are midpoints of
//     neighbouring levels, levels are conditional means of their cells,
//     (phi(t_k) - phi(t_k+1)) / (Phi(t_k+1) - Phi(t_k)) with t_K+1 = inf;
//     Lloyd's iteration from the uniform levels k 6/(2K+1) until no level
//     moves by more than 1e-15.
int quant_table(int kind, int bits, float* out) {
    if (bits != 2 && bits != 4) return 0;
    const int K = kmax_of_bits(bits);
    double t[8];
    if (kind == TDE_QUANT_MULAW) {
        const double mu = 255.0;
        for (int k = 1; k <= K; ++k) t[k - 1] = 3.0 * (std::pow(1.0 + mu, (k - 0.5) / (K + 0.5)) - 1.0) / mu;
    } else if (kind == TDE_QUANT_GAUSS) {
        auto pdf = [](double a) { return std::exp(-0.5 * a * a) / std::sqrt(2.0 * M_PI); };
        auto cdf = [](double a) { return 0.5 * std::erfc(-a / std::sqrt(2.0)); };
        double y[8];
        y[0] = 0.0;
        for (int k = 1; k <= K; ++k) y[k] = k * 6.0 / (2 * K + 1);
        for (int it = 0; it < 100000; ++it) {
            double b[8], ny[8];
            for (int k = 1; k <= K; ++k) b[k] = (y[k - 1] + y[k]) / 2.0;
            ny[0] = 0.0;
            double moved = 0.0;
            for (int k = 1; k <= K; ++k) {
                ny[k] = k < K ? (pdf(b[k]) - pdf(b[k + 1])) / (cdf(b[k + 1]) - cdf(b[k]))
                              : pdf(b[k]) / (1.0 - cdf(b[k]));
                moved = std::max(moved, std::fabs(ny[k] - y[k]));
            }
            for (int k = 1; k <= K; ++k) y[k] = ny[k];
            if (moved <= 1e-15) break;
        }
        for (int k = 1; k <= K; ++k) t[k - 1] = (y[k - 1] + y[k]) / 2.0;
    } else {
        return 0;
    }
    for (int k = 0; k < K; ++k) out[k] = (float)(t[k] * (2 * K + 1) / 6.0);
    return K;
}

// Doubles of scratch for the sum tree of an n-sample signal (block sums and
// the chunk sums of every further pass).
int64_t quantize_gsum_doubles(int64_t n) {
    int64_t len = (n + kSumBlock - 1) / kSumBlock, tot = len;
    while (len > 1) {
        len = (len + kSumChunk - 1) / kSumChunk;
        tot += len;
    }
    return tot + 1;
}

int launch_quantize(const QSig* sigs_dev, const QSig& one, int nsig, int64_t total_blocks, bool need_scale,
                    bool write_flags, int* zero_me, int nzero, hipStream_t s, int64_t min_n, int64_t max_n) {
    // short signals: the quantize blocks finish the sum tree themselves, and
    // the finalize kernel (one small launch) is left out
    // (large batches keep the finalize: one small launch costs less than every
    // block re-deriving its signal's scale)
    const int fused = need_scale && min_n >= 1 && max_n <= kFuseMaxN && total_blocks <= kFuseMaxBlocks ? 1 : 0;
    // equal lengths: the block -> signal map is a division (checked against
    // the grid, which is the sum of every signal's blocks)
    int bps = 0;
    if (sigs_dev && min_n >= 1 && min_n == max_n && total_blocks == nsig * ceil_div(min_n, kQuantBlock))
        bps = (int)ceil_div(min_n, kQuantBlock);
    if (need_scale) {
        hipLaunchKernelGGL(k_sumsq_blocks, dim3((unsigned)total_blocks), dim3(256), 0, s, sigs_dev, nsig, one, bps,
                           fused, zero_me, nzero);
    }
    if (!fused &&
        (need_scale || sigs_dev != nullptr || one.stat != nullptr || one.inv_out != nullptr || zero_me != nullptr))
        hipLaunchKernelGGL(k_scale_finalize, dim3(nsig), dim3(256), 0, s, sigs_dev, nsig, one, zero_me, nzero);
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)total_blocks), dim3(256), 0, s, sigs_dev, nsig, one, bps, fused);
    if (write_flags)
        hipLaunchKernelGGL(k_quantize_flags, dim3((unsigned)ceil_div(nsig, 256)), dim3(256), 0, s, sigs_dev, nsig,
                           one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
