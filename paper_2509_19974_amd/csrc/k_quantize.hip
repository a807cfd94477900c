// Algorithm 1, quantization step: per-signal scale and monotone integer quantization.
//
// Scale: S = sum of x^2 over the finite samples is an exact real (the
// quantizer on [-3 sigma, 3 sigma] fixes no summation order); the scale is
// sigma = sqrt(fl64(S) / n), inv_step = fl32((2K+1) / (6 sigma)) with fl64(S)
// the exact S rounded once. The kernels add the squares (each exact in
// float64) in float64 over a binary tree: pairs inside a lane, then across
// the wave that holds a 1024-sample node, then across nodes. That sum S' satisfies
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
// The kernels are HBM-bound: 4 bytes of x are read once for the scale and
// once for the codes; 1 byte of q, or the packed FP codes (4 or 6 bits) and
// the decimated input, are written. Whole blocks take a path without
// per-sample bounds checks. Keeping a block's samples on chip between the
// scale and the codes (one read) needs every block of a signal to wait for
// the signal's sum; a persistent one-pass kernel built that way measured
// slower than the two passes (the waits put several memory round trips on
// each workgroup's path, and its stash allows 3 to 4 workgroups per CU).
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

// Global-memory views of the descriptors' pointers: global loads and stores
// wait on the vector counter alone, where generic (flat) accesses also hold up
// every wait for the descriptors' scalar loads.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// 16 bytes of global memory (p 16-byte aligned) as a float4.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gload4(const float* p) {
    const f32x4_t v = *gmem(reinterpret_cast<const f32x4_t*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// The samples of block lb held by this thread: base + 1024 w + 256 k + 4 l + e
// for wave w, lane l and k, e < 4. Wave w holds node w of the block (1024
// samples) and each of its loads reads 1 KiB of consecutive samples; lanes
// 4j .. 4j+3 hold 16 consecutive samples.
__device__ __forceinline__ int64_t sample_of(int64_t lb, int k) {
    return lb * kQuantBlock + 1024 * (int64_t)(threadIdx.x >> 6) + 256 * k + 4 * (int64_t)(threadIdx.x & 63);
}

// This thread's 16 samples of block lb (sample_of), zero beyond n.
__device__ __forceinline__ void load_block(const QSig& s, int64_t lb, float4 (&xv)[4]) {
    if (lb * kQuantBlock + kQuantBlock <= s.n && ((((uintptr_t)s.x) & 15) == 0)) {
        // a whole aligned block (the workgroup's branch): four plain loads
#pragma unroll
        for (int k = 0; k < 4; ++k) xv[k] = gload4(s.x + sample_of(lb, k));
        return;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t m = sample_of(lb, k);
        if (m + 4 <= s.n && ((((uintptr_t)(s.x + m)) & 15) == 0)) {
            xv[k] = gload4(s.x + m);
        } else {
            float t4[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) t4[e] = (m + e < s.n) ? *gmem(s.x + m + e) : 0.f;
            xv[k] = make_float4(t4[0], t4[1], t4[2], t4[3]);
        }
    }
}

// Lane exchanges inside rows of 16 lanes (DPP), for 32- and 64-bit values.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = dpp_u32<CTRL>((uint32_t)b), hi = dpp_u32<CTRL>((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]: lane l ^ 1
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]: lane l ^ 2
constexpr int kDppNext = 0xF9;        // quad_perm [1,2,3,3]: lane l + 1 inside a quad
constexpr int kDppHalfMirror = 0x141; // lane 7 - i inside each 8 lanes
constexpr int kDppMirror = 0x140;     // lane 15 - i inside each 16 lanes

// The node sum of this wave's 1024 samples (load_block) in every lane: the
// squares (exact in float64) added pairwise inside the lane, then across
// quads, 8- and 16-lane groups (DPP) and the wave's 16- and 32-lane halves.
// Every level adds two equal-sized disjoint groups, so the whole is a binary
// tree of height 10 (a partner's sum is the same in both lanes: addition
// commutes).
__device__ __forceinline__ double wave_node_sum(const float4 (&xv)[4]) {
    double p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        p[k] = (sq_or_zero(xv[k].x) + sq_or_zero(xv[k].y)) + (sq_or_zero(xv[k].z) + sq_or_zero(xv[k].w));
    double a = (p[0] + p[1]) + (p[2] + p[3]);
    a = a + dpp_f64<kDppXor1>(a);
    a = a + dpp_f64<kDppXor2>(a);
    a = a + dpp_f64<kDppHalfMirror>(a);
    a = a + dpp_f64<kDppMirror>(a);
    a = a + __shfl_xor(a, 16, 64);
    a = a + __shfl_xor(a, 32, 64);
    return a;
}

// One block per 4096 samples of a signal: four level-10 nodes of the tree
// (1024 samples each), wave w summing node w.
// With the scale fused into the quantize kernel, this kernel also zeroes the
// statistics that kernel accumulates (first block of each signal) and the
// scratch counters of a later kernel (first block).
__global__ void __launch_bounds__(256) k_sumsq_blocks(const QSig* __restrict__ sigs, int nsig, QSig one, int bps, int fused,
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
    float4 xv[4];
    load_block(s, lb, xv);
    const double a = wave_node_sum(xv);
    if ((threadIdx.x & 63) == 0) {
        const int64_t node = lb * 4 + (threadIdx.x >> 6);
        if (node * kSumBlock < s.n) s.gsum[node] = a;
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
__device__ __attribute__((noinline)) double exact_sumsq_wg(const float* x, int64_t n) {
    __shared__ unsigned long long acc[kExactLimbs];
    __shared__ double res;
    for (int i = threadIdx.x; i < kExactLimbs; i += blockDim.x) acc[i] = 0ull;
    lds_barrier();
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
    lds_barrier();
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
    lds_barrier();
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
__global__ void __launch_bounds__(256) k_scale_finalize(const QSig* __restrict__ sigs, int nsig, QSig one, int* zero_me,
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

// Packed FP4/FP6 codes of one k: lanes 4j .. 4j+3 hold the 16 samples of one
// unit (4 each); a lane joins its bits with its right neighbour's to form
// the unit's dwords. m: the lane's first sample.
__device__ __forceinline__ void store_packed(const QSig& s, int64_t m, uint32_t w) {
    const int W = __builtin_amdgcn_readfirstlane(s.pk_bits);     // uniform
    const uint32_t z = W == 6 ? fp_bits4<6>(fp_bytes<6>(w)) : fp_bits4<4>(fp_bytes<4>(w));
    const uint32_t nb = dpp_u32<kDppNext>(z);
    const int j = threadIdx.x & 3;
    const int64_t unit = (m - 4 * j) / 16;
    if (16 * unit >= s.n) return;
    if (W == 6) {
        if (j == 0) *gmem(s.pk + 3 * unit) = z | (nb << 24);
        else if (j == 1) *gmem(s.pk + 3 * unit + 1) = (z >> 8) | (nb << 16);
        else if (j == 2) *gmem(s.pk + 3 * unit + 2) = (z >> 16) | (nb << 8);
    } else if (j == 0 || j == 2) {
        *gmem(s.pk + 2 * unit + (j >> 1)) = z | (nb << 16);
    }
}

// Decimated input of one k: the mean of 16 samples = 4 neighbouring lanes,
// summed ((x0+x1)+(x2+x3)) per lane, then lanes l^1, l^2 (the order of the
// stand-alone decimation kernel), times the scale.
__device__ __forceinline__ void store_dec(const QSig& s, int64_t m, const float4& x, float scale) {
    float a = (x.x + x.y) + (x.z + x.w);
    a += dpp_f32<kDppXor1>(a);
    a += dpp_f32<kDppXor2>(a);
    if ((threadIdx.x & 3) == 0 && m + 16 <= s.n) *gmem(s.dec + (m >> 4)) = f2bf_rne(a * (1.f / 16.f) * scale);
}

// quant_block for any block: every sample checked against n, any map.
__device__ __forceinline__ void quant_block_checked(const QSig& s, int64_t lb, const float4 (&xv)[4], float inv,
                                                    int K, long long& nonfinite_w, long long& nzero_w, int& sq,
                                                    int& sq2) {
    int nonfinite = 0, nzero = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t m = sample_of(lb, k);
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
                    *gmem(reinterpret_cast<uint32_t*>(s.q + m)) = w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (m + e < s.n) *gmem(s.q + m + e) = (int8_t)(w >> (8 * e));
                }
            }
        }
        if (s.pk) store_packed(s, m, w);
    }
    nonfinite_w = wave_sum<long long>(nonfinite);
    nzero_w = wave_sum<long long>(nzero);
}

// Codes of block lb from its samples (load_block) under scale inv: the int8
// codes, the packed FP codes and the decimated input where the descriptor asks
// for them, and one set of statistic atomics. Every thread of the workgroup
// calls it (a barrier inside when the signal has statistics).
//
// A whole block with the uniform map (or the sign map) takes a path without
// per-sample bounds checks: its counts come from wave ballots. Other blocks
// check every sample against n.
__device__ __forceinline__ void quant_block(const QSig& s, int64_t lb, const float4 (&xv)[4], float inv) {
    const int K = s.bits == 1 ? 1 : (1 << (s.bits - 1)) - 1;
    const bool want_sums = s.stat && !s.stat_lite;
    long long nonfinite_w, nzero_w;     // the wave's counts
    int sq = 0, sq2 = 0;                // the lane's sums (want_sums)
    if (s.dec) {
        const float scale = inv * s.dec_mul;
#pragma unroll
        for (int k = 0; k < 4; ++k) store_dec(s, sample_of(lb, k), xv[k], scale);
    }
    // the descriptor is uniform; reading its fields through the first lane
    // makes the branches below scalar ones
    const int bits = __builtin_amdgcn_readfirstlane(s.bits);
    const bool whole = __builtin_amdgcn_readfirstlane(
        lb * kQuantBlock + kQuantBlock <= s.n && s.nthr == 0 && (bits == 1 || inv > 0.f) &&
        (s.skip_q || ((((uintptr_t)s.q) & 3) == 0)));
    if (whole) {
        const bool store_q = !__builtin_amdgcn_readfirstlane(s.skip_q);
        const bool store_pk = __builtin_amdgcn_readfirstlane(s.pk != nullptr);
        const float Kf = (float)K;
        uint32_t nz = 0, nf = 0;        // wave counts (uniform)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t m = sample_of(lb, k);
            const float xs[4] = {xv[k].x, xv[k].y, xv[k].z, xv[k].w};
            int c[4];
            if (bits == 1) {
#pragma unroll
                for (int e = 0; e < 4; ++e) c[e] = (xs[e] > 0.f) - (xs[e] < 0.f);   // 0 for +-0 and NaN
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float r = __builtin_amdgcn_fmed3f(__builtin_rintf(__fmul_rn(xs[e], inv)), -Kf, Kf);
                    c[e] = xs[e] == xs[e] ? (int)r : 0;              // NaN -> 0, +-inf -> +-K
                }
            }
            uint32_t w = 0u;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                nf += (uint32_t)__builtin_popcountll(__ballot(!__builtin_isfinite(xs[e])));
                nz += (uint32_t)__builtin_popcountll(__ballot(c[e] == 0));
                if (want_sums) {
                    sq += c[e];
                    sq2 += c[e] * c[e];
                }
                w |= (uint32_t)(c[e] & 0xff) << (8 * e);
            }
            if (store_q) *gmem(reinterpret_cast<uint32_t*>(s.q + m)) = w;
            if (store_pk) store_packed(s, m, w);
        }
        nonfinite_w = nf;
        nzero_w = nz;
    } else {
        quant_block_checked(s, lb, xv, inv, K, nonfinite_w, nzero_w, sq, sq2);
    }
    if (s.stat) {
        __shared__ long long red[4][4];
        long long q1 = want_sums ? wave_sum<long long>(sq) : 0;
        long long q2 = want_sums ? wave_sum<long long>(sq2) : 0;
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[wv][0] = nonfinite_w; red[wv][1] = nzero_w; red[wv][2] = q1; red[wv][3] = q2;
        }
        lds_barrier();
        if (threadIdx.x < 4) {
            long long v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
            int64_t* dst = threadIdx.x == 0 ? &s.stat->n_nonfinite
                           : threadIdx.x == 1 ? &s.stat->n_zero
                           : threadIdx.x == 2 ? &s.stat->sum_q : &s.stat->sum_q2;
            if (v) atomicAdd((unsigned long long*)dst, (unsigned long long)v);
        }
    }
}

// 256 threads x 16 samples per block; one set of statistic atomics per block.
// fused: every block takes its signal's scale from the block sums itself
// (signals of 1 .. kFuseMaxN samples), and the first block of each signal
// publishes it.
template <bool fused>
__global__ void __launch_bounds__(256) k_quantize(const QSig* __restrict__ sigs, int nsig, QSig one, int bps) {
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
    } else if constexpr (fused) {
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
    float4 xv[4];
    load_block(s, lb, xv);
    quant_block(s, lb, xv, inv);
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
    if (fused)
        hipLaunchKernelGGL(k_quantize<true>, dim3((unsigned)total_blocks), dim3(256), 0, s, sigs_dev, nsig, one, bps);
    else
        hipLaunchKernelGGL(k_quantize<false>, dim3((unsigned)total_blocks), dim3(256), 0, s, sigs_dev, nsig, one, bps);
    if (write_flags)
        hipLaunchKernelGGL(k_quantize_flags, dim3((unsigned)ceil_div(nsig, 256)), dim3(256), 0, s, sigs_dev, nsig,
                           one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
