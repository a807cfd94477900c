// Exact sums of products of float32 values.
//
// Two quantities of the method are exact reals with no summation order: the
// sum of squares S = sum x^2 behind the quantizer's scale on [-3 sigma,
// 3 sigma], and the real correlation of Eq. (1) at the tied lags that the
// tie-refinement step of Algorithm 1 compares. The kernels first add them in
// float64 over a binary tree and keep that result when its rigorous error
// bound decides the outcome; otherwise they form the exact sum here.
//
// A finite float32 a is A 2^(ea - 150) with A < 2^24 an integer and ea >= 1
// (ea = 1 for subnormals), so a product a b is the integer A B < 2^48 times
// 2^(s - 298) with s = ea + eb - 2 in [0, 506]. A sum of at most 2^31 such
// terms is an integer multiple of 2^-298 below 2^585 in magnitude: it is held
// as kExactLimbs base-2^32 digits in int64 limbs, value sum limb[i] 2^(32 i - 298).
// Limbs may hold any int64 while terms are added; normalisation leaves
// limbs 0 .. kExactLimbs-2 in [0, 2^32) and the top limb signed (two's
// complement sense), so normalised sums compare digit by digit.
#pragma once

#include <stdint.h>

namespace tde {

constexpr int kExactLimbs = 20;

struct ExactTerm {
    uint64_t mag;    // A B < 2^48 (0 for a zero product)
    int shift;       // s = ea + eb - 2, in [0, 506]
    int neg;         // sign of the product
};

__host__ __device__ inline void exact_split(float f, uint32_t& m, int& e, uint32_t& sgn) {
    const uint32_t b = __builtin_bit_cast(uint32_t, f);
    sgn = b >> 31;
    const uint32_t E = (b >> 23) & 0xffu;
    m = E ? ((b & 0x7fffffu) | 0x800000u) : (b & 0x7fffffu);
    e = E ? (int)E : 1;
}

// the product a b of two finite float32 values as an exact term
__host__ __device__ inline ExactTerm exact_term(float a, float b) {
    uint32_t ma, mb, sa, sb;
    int ea, eb;
    exact_split(a, ma, ea, sa);
    exact_split(b, mb, eb, sb);
    ExactTerm t;
    t.mag = (uint64_t)ma * (uint64_t)mb;
    t.shift = ea + eb - 2;
    t.neg = (int)(sa ^ sb);
    return t;
}

// The three base-2^32 digits (lo, mid, hi) of mag 2^(shift mod 32), which
// start at limb shift / 32.
__host__ __device__ inline void exact_digits(const ExactTerm& t, int& limb, uint32_t& lo, uint32_t& mid,
                                             uint32_t& hi) {
    const int off = t.shift & 31;
    limb = t.shift >> 5;
    lo = (uint32_t)(t.mag << off);
    const uint64_t up = off ? (t.mag >> (32 - off)) : (t.mag >> 32);   // (mag << off) >> 32
    mid = (uint32_t)up;
    hi = (uint32_t)(up >> 32);
}

// Carries upward: limbs 0 .. kExactLimbs-2 end in [0, 2^32), the top limb
// keeps the sign. Arithmetic shifts make the carry the floor quotient.
__host__ __device__ inline void exact_normalize(int64_t* limb) {
    for (int i = 0; i < kExactLimbs - 1; ++i) {
        const int64_t c = limb[i] >> 32;
        limb[i] -= c * ((int64_t)1 << 32);
        limb[i + 1] += c;
    }
}

// Order of two normalised sums: -1, 0 or +1 for a < b, a == b, a > b.
__host__ __device__ inline int exact_compare(const int64_t* a, const int64_t* b) {
    if (a[kExactLimbs - 1] != b[kExactLimbs - 1]) return a[kExactLimbs - 1] < b[kExactLimbs - 1] ? -1 : 1;
    for (int i = kExactLimbs - 2; i >= 0; --i)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

// A normalised sum rounded once to float64, round to nearest, ties to even
// (every value it can hold, 2^-298 .. 2^585, is a normal float64 or 0).
__host__ __device__ inline double exact_to_double(const int64_t* limb_in) {
    int64_t v[kExactLimbs];
    const bool neg = limb_in[kExactLimbs - 1] < 0;
    for (int i = 0; i < kExactLimbs; ++i) v[i] = neg ? -limb_in[i] : limb_in[i];
    if (neg) exact_normalize(v);
    int h = kExactLimbs - 1;
    while (h >= 0 && v[h] == 0) --h;
    if (h < 0) return 0.0;
    const uint64_t d2 = (uint64_t)v[h];
    const uint64_t d1 = h >= 1 ? (uint64_t)v[h - 1] : 0u;
    const uint64_t d0 = h >= 2 ? (uint64_t)v[h - 2] : 0u;
    bool sticky = false;
    for (int i = 0; i < h - 2; ++i) sticky |= v[i] != 0;
    const int p = 63 - __builtin_clzll(d2);            // top bit of d2, 0 .. 31 (bit 64 + p of the window)
    // the 64 bits below and at the window's top bit
    const uint64_t w = (d2 << (63 - p)) | (d1 << (31 - p)) | (d0 >> (p + 1));
    sticky |= (d0 & ((((uint64_t)1) << (p + 1)) - 1u)) != 0;
    uint64_t mant = w >> 11;                           // 53 bits
    const uint64_t rest = w & 0x7ffu;
    if (rest > 0x400u || (rest == 0x400u && (sticky || (mant & 1u)))) ++mant;
    // weight of the window's top bit: 2^(32 h + p - 298); of mant's last bit 52 below
    int e = 32 * h + p - 298 - 52;
    if (mant >> 53) {
        mant >>= 1;
        ++e;
    }
    double r = (double)mant;
    // exact scaling by 2^e in at most three steps (each factor a normal power of two)
    while (e > 0) {
        const int k = e > 1000 ? 1000 : e;
        r *= __builtin_bit_cast(double, (uint64_t)(1023 + k) << 52);
        e -= k;
    }
    while (e < 0) {
        const int k = e < -1000 ? 1000 : -e;
        r *= __builtin_bit_cast(double, (uint64_t)(1023 - k) << 52);
        e += k;
    }
    return neg ? -r : r;
}

// Relative error bound of a float64 sum of non-negative terms (or of the
// absolute values of signed ones) formed over any binary tree of height at
// most 64 (every sum of at most 2^64 terms): |computed - exact| <= gamma_64
// sum |t|, gamma_64 = 64 u / (1 - 64 u), u = 2^-53 (Higham, Accuracy and
// Stability of Numerical Algorithms, 2nd ed., Section 4.2). The constant
// 2^-45 = 256 u is more than twice that, which also covers the rounding of
// the bound's own arithmetic.
constexpr double kTreeRelErr = 2.8421709430404007e-14;   // 2^-45

}  // namespace tde
