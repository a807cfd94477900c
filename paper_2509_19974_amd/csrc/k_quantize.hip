// Algorithm 1, lines 1-2: per-signal scale and monotone integer quantization.
//
// Scale: S = sum of x^2 over finite samples, every square exact in float64,
// summed in float64 in a fixed order (groups of 256 consecutive values summed
// left to right; the group sums grouped the same way until one value is
// left). sigma = sqrt(S / n), inv_step = fl32((2K+1) / (6 sigma)).
//
// Quantizer: bits = 1 is sign with sign(0) = 0 (Section 4.2), taken from the
// IEEE bits; bits in {2,4,8} is clamp(round_half_even(fl32(x * inv_step)),
// -K, K). Both are monotone non-decreasing with phi(0) = 0 (Theorem 1).
//
// The three kernels are HBM-bound: 4 bytes of x are read once for the scale
// and once for the codes, 1 byte of q is written.
#include "tde_internal.h"

namespace tde {

constexpr int kFanIn = 256;       // sum-tree fan-in (part of the scale's definition)

__device__ __forceinline__ const QSig& pick_sig(const QSig* sigs, int nsig, const QSig& one,
                                                int64_t unit, bool by_group, int64_t& local) {
    if (sigs == nullptr) {
        local = unit;
        return one;
    }
    // binary search: last signal whose base <= unit
    int lo = 0, hi = nsig - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int64_t b = by_group ? sigs[mid].grp_base : sigs[mid].blk_base;
        if (b <= unit) lo = mid; else hi = mid - 1;
    }
    local = unit - (by_group ? sigs[lo].grp_base : sigs[lo].blk_base);
    return sigs[lo];
}

// One thread per group of 256 samples: the group's left-to-right float64 sum.
__global__ void __launch_bounds__(256) k_sumsq_groups(const QSig* sigs, int nsig, QSig one,
                                                      int64_t total_groups) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_groups) return;
    int64_t lg;
    const QSig& s = pick_sig(sigs, nsig, one, g, true, lg);
    if (s.inv_fixed > 0.f || s.bits == 1) return;
    int64_t lo = lg * kFanIn;
    int64_t hi = lo + kFanIn < s.n ? lo + kFanIn : s.n;
    const float* x = s.x;
    double acc = 0.0;
    int64_t m = lo;
    if ((((uintptr_t)(x + m)) & 15) == 0) {
        // 16 independent loads in flight, then the left-to-right additions
        for (; m + 64 <= hi; m += 64) {
            float4 f[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) f[k] = *reinterpret_cast<const float4*>(x + m + 4 * k);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                double a0 = f[k].x, a1 = f[k].y, a2 = f[k].z, a3 = f[k].w;
                acc += __builtin_isfinite(a0) ? a0 * a0 : 0.0;
                acc += __builtin_isfinite(a1) ? a1 * a1 : 0.0;
                acc += __builtin_isfinite(a2) ? a2 * a2 : 0.0;
                acc += __builtin_isfinite(a3) ? a3 * a3 : 0.0;
            }
        }
    }
    for (; m < hi; ++m) {
        double a = x[m];
        acc += __builtin_isfinite(a) ? a * a : 0.0;
    }
    s.gsum[lg] = acc;
}

// One block per signal: remaining levels of the sum tree, then the scale.
// Also zeroes the statistics that the quantize kernel accumulates.
__global__ void __launch_bounds__(256) k_scale_finalize(const QSig* sigs, int nsig, QSig one) {
    const QSig& s = sigs ? sigs[blockIdx.x] : one;
    const int t = threadIdx.x;
    float inv;
    if (s.bits == 1) {
        inv = 0.f;
    } else if (s.inv_fixed > 0.f) {
        inv = s.inv_fixed;
    } else {
        // levels >= 1: each level's sums are written after the previous level
        // in the same scratch (sized by quantize_gsum_doubles), so no thread
        // overwrites values another thread still reads.
        int64_t len = (s.n + kFanIn - 1) / kFanIn;
        double* a = s.gsum;
        double* out = a + len;
        while (len > 1) {
            int64_t nn = (len + kFanIn - 1) / kFanIn;
            for (int64_t g = t; g < nn; g += blockDim.x) {
                int64_t lo = g * kFanIn;
                int64_t hi = lo + kFanIn < len ? lo + kFanIn : len;
                double acc = 0.0;
                int64_t i = lo;
                for (; i + 16 <= hi; i += 16) {
                    double v[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) v[k] = a[i + k];
#pragma unroll
                    for (int k = 0; k < 16; ++k) acc += v[k];
                }
                for (; i < hi; ++i) acc += a[i];
                out[g] = acc;
            }
            __syncthreads();
            a = out;
            out = a + nn;
            len = nn;
        }
        double S = a[0];
        if (S > 0.0) {
            int K = (1 << (s.bits - 1)) - 1;
            double var = S / (double)s.n;
            double sigma = __builtin_sqrt(var);
            double v = (double)(2 * K + 1) / (6.0 * sigma);
            inv = (float)v;
        } else {
            inv = 0.f;
        }
    }
    if (t == 0) {
        if (s.inv_out) *s.inv_out = inv;
        if (s.stat) {
            s.stat->inv_step = inv;
            s.stat->flags = 0;
            s.stat->n_nonfinite = 0;
            s.stat->n_zero = 0;
            s.stat->sum_q = 0;
            s.stat->sum_q2 = 0;
        }
    }
}

__device__ __forceinline__ int quant1(float xf, int bits, float inv, int K, int& nonfinite) {
    uint32_t b = __float_as_uint(xf);
    uint32_t mag = b & 0x7fffffffu;
    bool is_nan = mag > 0x7f800000u;
    nonfinite += (mag >= 0x7f800000u) ? 1 : 0;
    if (bits == 1) {
        if (is_nan || mag == 0) return 0;
        return (b >> 31) ? -1 : 1;
    }
    if (is_nan || inv == 0.f) return 0;
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
__global__ void __launch_bounds__(256) k_quantize(const QSig* sigs, int nsig, QSig one,
                                                  int64_t total_blocks) {
    int64_t blk = blockIdx.x;
    int64_t lb;
    const QSig& s = pick_sig(sigs, nsig, one, blk, false, lb);
    const float inv = (s.bits == 1) ? 0.f : (s.inv_fixed > 0.f ? s.inv_fixed : *s.inv_out);
    const int K = s.bits == 1 ? 1 : (1 << (s.bits - 1)) - 1;
    const int64_t m0 = lb * kQuantBlock + 16 * (int64_t)threadIdx.x;
    int nonfinite = 0, nzero = 0;
    int sq = 0, sq2 = 0;
    if (m0 < s.n) {
        float xs[16];
        const bool full = m0 + 16 <= s.n;
        if (full && ((((uintptr_t)(s.x + m0)) & 15) == 0)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float4 f = *reinterpret_cast<const float4*>(s.x + m0 + 4 * k);
                xs[4 * k] = f.x; xs[4 * k + 1] = f.y; xs[4 * k + 2] = f.z; xs[4 * k + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) xs[e] = (m0 + e < s.n) ? s.x[m0 + e] : 0.f;
        }
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int c = quant1(xs[e], s.bits, inv, K, nonfinite);
            if (m0 + e < s.n) {
                nzero += c == 0;
                sq += c;
                sq2 += c * c;
            }
            w[e >> 2] |= (uint32_t)(uint8_t)c << (8 * (e & 3));
        }
        if (full && ((((uintptr_t)(s.q + m0)) & 15) == 0)) {
            *reinterpret_cast<uint4*>(s.q + m0) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                if (m0 + e < s.n) s.q[m0 + e] = (int8_t)(w[e >> 2] >> (8 * (e & 3)));
        }
    }
    if (s.stat) {
        __shared__ long long red[4][4];
        long long a = wave_sum<long long>(nonfinite);
        long long z = wave_sum<long long>(nzero);
        long long q1 = wave_sum<long long>(sq);
        long long q2 = wave_sum<long long>(sq2);
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

// Flags from the finished statistics (one thread per signal).
__global__ void k_quantize_flags(const QSig* sigs, int nsig, QSig one) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsig) return;
    const QSig& s = sigs ? sigs[i] : one;
    if (!s.stat) return;
    int f = 0;
    if (s.stat->n_nonfinite) f |= TDE_FLAG_NONFINITE_X;
    if (s.stat->n_zero == s.n) f |= TDE_FLAG_ZERO_X;
    s.stat->flags = f;
}

// Doubles of scratch for the sum tree of an n-sample signal (all levels).
int64_t quantize_gsum_doubles(int64_t n) {
    int64_t len = (n + kFanIn - 1) / kFanIn, tot = len;
    while (len > 1) {
        len = (len + kFanIn - 1) / kFanIn;
        tot += len;
    }
    return tot + 1;
}

int launch_quantize(const QSig* sigs_dev, const QSig& one, int nsig, int64_t total_groups,
                    int64_t total_blocks, bool need_scale, hipStream_t s) {
    if (need_scale) {
        hipLaunchKernelGGL(k_sumsq_groups, dim3((unsigned)ceil_div(total_groups, 256)), dim3(256), 0, s,
                           sigs_dev, nsig, one, total_groups);
    }
    if (need_scale || sigs_dev != nullptr || one.stat != nullptr || one.inv_out != nullptr)
        hipLaunchKernelGGL(k_scale_finalize, dim3(nsig), dim3(256), 0, s, sigs_dev, nsig, one);
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)total_blocks), dim3(256), 0, s, sigs_dev, nsig, one,
                       total_blocks);
    hipLaunchKernelGGL(k_quantize_flags, dim3((unsigned)ceil_div(nsig, 256)), dim3(256), 0, s, sigs_dev,
                       nsig, one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
