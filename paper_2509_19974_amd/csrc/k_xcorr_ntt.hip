// Algorithm 1, correlation step for long signals: the exact integer correlation as a
// cyclic convolution computed with number-theoretic transforms modulo one or
// two primes, combined by the Chinese remainder theorem (the multimodular
// route among the exact multiplication methods of Section 3.2).
//
// With ur = u reversed, (ur conv v)[j] = r[j - (nu - 1)]. A cyclic
// convolution of length n = 2^L equals the linear one at every position
// j in [jlo, jhi] when no other position aliases onto it; the host picks
// n > max(jhi, nu + nv - 2 - jlo). |r| <= overlap * Ku * Kv (the coefficient
// bound of Section 3.2): one prime suffices below p1 / 2, two primes
// (product ~ 2^59.4) cover every int8 case this library accepts (|r| <=
// 2^23 x 127^2 < 2^37).
//
// Transform (four-step, n = n1 x 4096, element j = b + 4096 i):
//   K1 columns:  for each column b, a length-n1 decimation-in-frequency
//                transform over i (output in bit-reversed order of k1),
//                then the factor w_n^(b k1);
//   K2 rows:     for each row (fixed k1), a length-4096 DIF transform over b
//                of both signals, the pointwise product, and the inverse
//                (decimation-in-time) row transform, all on chip;
//   K3 columns:  the factor w_n^(-b k1), the inverse length-n1 transform,
//                scaling by 1/n, CRT to a signed 64-bit value, the output r
//                and the (max, smallest index, count) triple of the tile.
// Arithmetic: primes below 2^30, so that residues may be kept lazily in
// [0, 2p) or [0, 4p) inside 32 bits. Butterflies multiply by a twiddle w
// with Shoup's method (the table holds w and floor(w 2^32 / p); the product
// lands in [0, 2p) with two low and one high 32-bit multiply). The forward
// (decimation-in-frequency) butterfly keeps its values in [0, 2p), the
// inverse (decimation-in-time) one in [0, 4p), as in Harvey's lazy
// butterflies. The pointwise product, the chained column factors and the
// final scaling use Montgomery multiplication with R = 2^32, which needs
// a b < p 2^32: every use has both factors below 2p, or one below p and
// the other below 4p, so a b < 4 p^2 < p 2^32.
// Twiddle tables hold plain residues with their Shoup quotients.
#include <algorithm>
#include <vector>

#include "tde_internal.h"

namespace tde {

namespace {

// 119 2^23 + 1 and 45 2^24 + 1: both below 2^30 (4p < 2^32), 2^23 divides
// p - 1 (transforms up to 2^23 points), and p1 < 2 p2 (one conditional
// subtraction reduces a residue mod p1 to one mod p2 in the CRT)
constexpr uint32_t kP[2] = {998244353u, 754974721u};
constexpr uint32_t kG[2] = {3u, 11u};                     // primitive roots

__device__ __forceinline__ uint32_t mont(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
    const uint32_t m = tlo * pinv;                 // t p^-1 mod 2^32
    const uint32_t mh = __umulhi(m, p);            // (t - m p) / 2^32 = thi - mh exactly
    const uint32_t r = thi - mh;
    return thi < mh ? r + p : r;
}

__device__ __forceinline__ uint32_t subm(uint32_t a, uint32_t b, uint32_t p) {
    return a >= b ? a - b : a + p - b;
}

__device__ __forceinline__ uint32_t residue(int8_t x, uint32_t p) {
    return x < 0 ? (uint32_t)((int32_t)p + x) : (uint32_t)x;
}

// a w mod p in [0, 2p) for any 32-bit a, from t = (w, floor(w 2^32 / p)), w < p
__device__ __forceinline__ uint32_t shoup(uint32_t a, uint2 t, uint32_t p) {
    const uint32_t q = __umulhi(a, t.y);
    return a * t.x - q * p;
}

// [0, 4p) -> [0, 2p): a - 2p wraps above a unless a >= 2p
__device__ __forceinline__ uint32_t red2(uint32_t a, uint32_t p2) {
    const uint32_t b = a - p2;
    return b < a ? b : a;
}

// forward butterfly, x, y in [0, 2p): (x + y, (x - y) w), both in [0, 2p)
__device__ __forceinline__ void dif(uint32_t& x, uint32_t& y, uint2 t, uint32_t p, uint32_t p2) {
    const uint32_t s = x + y, d = x + p2 - y;
    x = red2(s, p2);
    y = shoup(d, t, p);
}

// inverse butterfly, x, y in [0, 4p): (x + y w, x - y w), both in [0, 4p)
__device__ __forceinline__ void dit(uint32_t& x, uint32_t& y, uint2 t, uint32_t p, uint32_t p2) {
    const uint32_t a = red2(x, p2), b = shoup(y, t, p);
    x = a + b;
    y = a + p2 - b;
}

__device__ __forceinline__ uint32_t brev(uint32_t x, int bits) {
    return bits ? __builtin_bitreverse32(x) >> (32 - bits) : 0u;
}

// Column block of workgroup x of nb: workgroups are dealt to the 8 XCDs in
// turn, so x = 8 q + r takes block r (nb / 8) + q, and the blocks that one
// XCD works on at a time are neighbours (their short row segments share L2
// lines).
__device__ __forceinline__ int xcd_block(int x, int nb) {
    return (nb & 7) ? x : (x & 7) * (nb >> 3) + (x >> 3);
}

// table layout per prime, (w, Shoup quotient) pairs: TC[n1] (w_n1^k),
// TL[4096] (w_n^k), TR[4096] (w_4096^k)
__device__ __forceinline__ const uint2* tab_of(const NttGroup& g, int pr) {
    return reinterpret_cast<const uint2*>(g.tab) + (size_t)pr * (g.n1 + 2 * kNttRow);
}

// x w_n^e in [0, 2p) for e in [0, n): w_n^e = w_n1^(e >> 12) w_n^(e & 4095)
__device__ __forceinline__ uint32_t twist(uint32_t x, const uint2* T, int n1, uint32_t e, uint32_t p) {
    return shoup(shoup(x, T[n1 + (e & 4095u)], p), T[e >> 12], p);
}

// ------------------------------------------------------------- tables --

__global__ void k_ntt_tables(NttGroup g) {
    const int per = g.n1 + 2 * kNttRow;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)per * g.nprimes) return;
    const int pr = (int)(k / per);
    const int o = (int)(k % per);
    const uint32_t p = g.p[pr], pinv = g.pinv[pr];
    uint64_t e;                                    // exponent of w_n
    if (o < g.n1) e = (uint64_t)o << 12;
    else if (o < g.n1 + kNttRow) e = (uint64_t)(o - g.n1);
    else e = (uint64_t)(o - g.n1 - kNttRow) * (uint64_t)g.n1;
    uint32_t acc = g.one_m[pr], base = g.root_m[pr];
    while (e) {
        if (e & 1) acc = mont(acc, base, p, pinv);
        base = mont(base, base, p, pinv);
        e >>= 1;
    }
    const uint32_t w = mont(acc, 1u, p, pinv);   // out of Montgomery form
    reinterpret_cast<uint2*>(g.tab)[k] = make_uint2(w, (uint32_t)(((uint64_t)w << 32) / p));
}

// ------------------------------------------------- K1: forward columns --
// grid (4096 / kNttC1, 2 sides, njobs), every prime in turn; LDS: kNttC1 x n1 residues,
// row-major (16 consecutive columns of a row side by side).

__global__ void __launch_bounds__(1024) k_ntt_cols_fwd(NttGroup g, const NttJob* jobs) {
    extern __shared__ uint32_t L[];
    const NttJob& J = jobs[blockIdx.z];
    const int side = blockIdx.y;                   // 0: reversed u, 1: v
    const int n1 = g.n1, ln1 = g.log_n1;
    const int b0 = xcd_block(blockIdx.x, gridDim.x) * kNttC1;
    const int tot = kNttC1 * n1;
    const int8_t* src = side ? J.v : J.u;
    const int64_t nsrc = side ? J.nv : J.nu;
    // the thread's codes (elements threadIdx.x + 1024 m of the block), all
    // loads in flight together, kept for every prime
    int32_t code[kNttK1Per];
#pragma unroll
    for (int m = 0; m < kNttK1Per; ++m) {
        const int idx = threadIdx.x + m * 1024;
        int32_t v = 0;
        if (idx < tot) {
            const int c = idx % kNttC1, i = idx / kNttC1;
            const int64_t j = b0 + c + ((int64_t)i << 12);
            if (j < nsrc) v = side ? src[j] : src[nsrc - 1 - j];
        }
        code[m] = v;
    }
    for (int pr = 0; pr < g.nprimes; ++pr) {
        const uint32_t p = g.p[pr], p2 = 2 * p;
        const uint2* T = tab_of(g, pr);
        if (pr) lds_barrier();                         // the previous prime's residues are read
#pragma unroll
        for (int m = 0; m < kNttK1Per; ++m) {
            const int idx = threadIdx.x + m * 1024;
            if (idx < tot) L[idx] = residue((int8_t)code[m], p);
        }
        lds_barrier();
        // decimation in frequency over i: half-distance h = n1/2 .. 1, two
        // stages per pass through LDS (h and h/2 on the four rows r0 = base +
        // pos, r0 + h/2, r0 + h, r0 + 3h/2 of a 2h group: the same butterflies,
        // twiddles and order as one stage at a time), then a last single stage
        // when log2(n1) is odd
        int lh = ln1 - 1;
        // three stages per pass (h, h/2, h/4 on the eight rows base + pos +
        // k h/4 of a 2h group) while at least three remain
        for (; lh >= 2; lh -= 3) {
            const int h4 = 1 << (lh - 2);
            const int s1 = ln1 - 1 - lh;
            // the seven twiddles of a group at position pos: stage h (4), h/2 (2), h/4 (1)
            auto twiddles = [&](int pos, uint2(&w)[7]) {
#pragma unroll
                for (int k = 0; k < 4; ++k) w[k] = T[(pos + k * h4) << s1];
                w[4] = T[pos << (s1 + 1)];
                w[5] = T[(pos + h4) << (s1 + 1)];
                w[6] = T[pos << (s1 + 2)];
            };
            auto group = [&](int bi, const uint2(&w)[7]) {
                const int c = bi % kNttC1, q = bi / kNttC1;
                const int pos = q & (h4 - 1);
                uint32_t* x0 = &L[(((q >> (lh - 2)) << (lh + 1)) + pos) * kNttC1 + c];
                uint32_t x[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) x[k] = x0[k * h4 * kNttC1];
#pragma unroll
                for (int k = 0; k < 4; ++k) dif(x[k], x[k + 4], w[k], p, p2);              // stage h
#pragma unroll
                for (int k = 0; k < 8; k += (k & 1) ? 3 : 1)                               // stage h/2: k = 0, 1, 4, 5
                    dif(x[k], x[k + 2], w[4 + (k & 1)], p, p2);
#pragma unroll
                for (int k = 0; k < 8; k += 2) dif(x[k], x[k + 1], w[6], p, p2);           // stage h/4
#pragma unroll
                for (int k = 0; k < 8; ++k) x0[k * h4 * kNttC1] = x[k];
            };
            if (((int)blockDim.x / kNttC1) % h4 == 0) {
                // every group of this thread has the same position: twiddles once
                uint2 w[7];
                twiddles((int)(threadIdx.x / kNttC1) & (h4 - 1), w);
                for (int bi = threadIdx.x; bi < tot / 8; bi += blockDim.x) group(bi, w);
            } else {
                for (int bi = threadIdx.x; bi < tot / 8; bi += blockDim.x) {
                    uint2 w[7];
                    twiddles((bi / kNttC1) & (h4 - 1), w);
                    group(bi, w);
                }
            }
            lds_barrier();
        }
        if (lh == 1) {
            const int h = 1 << lh, h2 = h >> 1;
            const int s1 = ln1 - 1 - lh;             // twiddle index shift of stage h (stage h/2: s1 + 1)
            for (int bi = threadIdx.x; bi < tot / 4; bi += blockDim.x) {
                const int c = bi % kNttC1, q = bi / kNttC1;
                const int pos = q & (h2 - 1);
                const int r0 = ((q >> (lh - 1)) << (lh + 1)) + pos;
                uint32_t* x0 = &L[r0 * kNttC1 + c];
                uint32_t* x1 = x0 + h2 * kNttC1;
                uint32_t* x2 = x0 + h * kNttC1;
                uint32_t* x3 = x2 + h2 * kNttC1;
                uint32_t a0 = *x0, a1 = *x1, a2 = *x2, a3 = *x3;
                dif(a0, a2, T[pos << s1], p, p2);
                dif(a1, a3, T[(pos + h2) << s1], p, p2);
                const uint2 w2 = T[pos << (s1 + 1)];
                dif(a0, a1, w2, p, p2);
                dif(a2, a3, w2, p, p2);
                *x0 = a0;
                *x1 = a1;
                *x2 = a2;
                *x3 = a3;
            }
            lds_barrier();
            lh -= 2;
        }
        if (lh == 0) {
            for (int bi = threadIdx.x; bi < tot / 2; bi += blockDim.x) {
                const int c = bi % kNttC1, e = 2 * (bi / kNttC1);
                uint32_t a = L[e * kNttC1 + c], b = L[(e + 1) * kNttC1 + c];
                dif(a, b, T[0], p, p2);
                L[e * kNttC1 + c] = a;
                L[(e + 1) * kNttC1 + c] = b;
            }
            lds_barrier();
        }
        // factor w_n^(b k1), k1 = bit-reversed row index; store the residues
        uint32_t* out = J.res + ((size_t)side * g.nprimes + pr) * ((size_t)n1 << 12);
        if (ln1 >= 6) {
            // thread: column c, rows i = i0 + 64 m with k1 = K + brev(m), K =
            // brev6(i0) << (ln1 - 6); taking m in the order of brev(m) the
            // factor is f = w^(b K) times w^b per step, carried with one R
            // (Montgomery form) so that one Montgomery product applies it
            const int c = threadIdx.x & (kNttC1 - 1), i0 = threadIdx.x >> 4, lm = ln1 - 6;
            const uint32_t b = b0 + c;
            uint32_t f = twist(g.one_m[pr], T, n1, b * (brev((uint32_t)i0, 6) << lm), p);   // R w^(b K), [0, 2p)
            const uint2 step = T[n1 + b];                                                    // w_n^b
            for (int mr = 0; mr < (1 << lm); ++mr) {
                const int i = i0 + (int)(brev((uint32_t)mr, lm) << 6);
                out[(size_t)b + ((size_t)i << 12)] = mont(L[c + i * kNttC1], f, p, g.pinv[pr]);
                f = shoup(f, step, p);
            }
        } else {
            for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
                const int c = idx % kNttC1, i = idx / kNttC1;
                const uint32_t k1 = brev((uint32_t)i, ln1);
                const uint32_t e = (uint32_t)(b0 + c) * k1;          // < 4096 n1 = n <= 2^23
                out[(size_t)b0 + c + ((size_t)i << 12)] = twist(L[idx], T, n1, e, p);
            }
        }
    }
}

// ---------------------------------------------------- K2: fused rows --
// grid (n1, nprimes, njobs), 256 threads, 16 residues per thread.
// Rounds of 4 radix-2 stages in registers with LDS exchanges between them:
//   round A: elements t + 256 k   (h = 2048 .. 256)
//   round B: elements 256 (t/16) + t%16 + 16 k   (h = 128 .. 16)
//   round C: elements 16 t + k    (h = 8 .. 1)
// LDS index b + b/16 keeps the exchanges free of bank conflicts.

__device__ __forceinline__ int rpos(int round, int t, int k) {
    if (round == 0) return t + 256 * k;
    if (round == 1) return ((t >> 4) << 8) + (t & 15) + 16 * k;
    return 16 * t + k;
}

__device__ __forceinline__ int lds_ix(int b) { return b + (b >> 4); }

// Twiddles of a round. At the stage with register distance d = 2^ld (row
// half-distance 2^lh, lh = ld + 8, 4, 0 in rounds A, B, C) element k of
// thread t takes w_4096^e, e = (rpos mod 2^(lh+1)) << (11 - lh); for the
// upper element's partner k (bit ld clear) e splits into a lane part
// lane(round, t) << (11 - lh) and (k mod d) << (11 - ld), which is the same
// in every lane. The lane part's twiddle is one load per stage; the other
// comes from a lane-uniform load, and the butterfly multiplies by both
// (once when either is 1).
__device__ __forceinline__ int lane_part(int round, int t) { return round == 0 ? t : (round == 1 ? (t & 15) : 0); }

__device__ __forceinline__ void dif2(uint32_t& x, uint32_t& y, uint2 a, uint2 b, uint32_t p, uint32_t p2) {
    const uint32_t s = x + y, d = x + p2 - y;
    x = red2(s, p2);
    y = shoup(shoup(d, a, p), b, p);
}

__device__ __forceinline__ void dit2(uint32_t& x, uint32_t& y, uint2 a, uint2 b, uint32_t p, uint32_t p2) {
    const uint32_t u = red2(x, p2), v = shoup(shoup(y, a, p), b, p);
    x = u + v;
    y = u + p2 - v;
}

// forward DIF stages of one round (h decreasing)
__device__ __forceinline__ void dif_round(uint32_t* x, int round, int t, const uint2* TR, uint32_t p) {
    const int lstride = round == 0 ? 8 : (round == 1 ? 4 : 0);
#pragma unroll
    for (int ld = 3; ld >= 0; --ld) {
        const int d = 1 << ld;
        const int lh = ld + lstride;
        const uint2 A = TR[lane_part(round, t) << (11 - lh)];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k & d) continue;
            const int ku = k & (d - 1);
            if (round == 2) dif(x[k], x[k + d], TR[ku << (11 - ld)], p, 2 * p);
            else if (ku == 0) dif(x[k], x[k + d], A, p, 2 * p);
            else dif2(x[k], x[k + d], A, TR[ku << (11 - ld)], p, 2 * p);
        }
    }
}

// inverse DIT stages of one round (h increasing), twiddles w^-e
__device__ __forceinline__ void dit_round(uint32_t* x, int round, int t, const uint2* TR, uint32_t p) {
    const int lstride = round == 0 ? 8 : (round == 1 ? 4 : 0);
#pragma unroll
    for (int ld = 0; ld <= 3; ++ld) {
        const int d = 1 << ld;
        const int lh = ld + lstride;
        const uint2 A = TR[(kNttRow - (lane_part(round, t) << (11 - lh))) & (kNttRow - 1)];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k & d) continue;
            const int ku = k & (d - 1);
            const uint2 B = TR[(kNttRow - (ku << (11 - ld))) & (kNttRow - 1)];
            if (round == 2) dit(x[k], x[k + d], B, p, 2 * p);
            else if (ku == 0) dit(x[k], x[k + d], A, p, 2 * p);
            else dit2(x[k], x[k + d], A, B, p, 2 * p);
        }
    }
}

__device__ __forceinline__ void exchange(uint32_t* x, uint32_t* S, int from, int to, int t) {
#pragma unroll
    for (int k = 0; k < 16; ++k) S[lds_ix(rpos(from, t, k))] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = S[lds_ix(rpos(to, t, k))];
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_ntt_rows(NttGroup g, const NttJob* jobs) {
    __shared__ uint32_t S[kNttRow + kNttRow / 16];
    const NttJob& J = jobs[blockIdx.z];
    const int pr = blockIdx.y;
    const uint32_t p = g.p[pr], pinv = g.pinv[pr];
    const uint2* __restrict__ TR = tab_of(g, pr) + g.n1 + kNttRow;
    const size_t n = (size_t)g.n1 << 12;
    uint32_t* U = J.res + (size_t)pr * n + ((size_t)blockIdx.x << 12);
    const uint32_t* V = J.res + ((size_t)g.nprimes + pr) * n + ((size_t)blockIdx.x << 12);
    const int t = threadIdx.x;
    uint32_t xu[16], xv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) xu[k] = U[t + 256 * k];
#pragma unroll
    for (int k = 0; k < 16; ++k) xv[k] = V[t + 256 * k];
    dif_round(xu, 0, t, TR, p);
    exchange(xu, S, 0, 1, t);
    dif_round(xu, 1, t, TR, p);
    exchange(xu, S, 1, 2, t);
    dif_round(xu, 2, t, TR, p);
    dif_round(xv, 0, t, TR, p);
    exchange(xv, S, 0, 1, t);
    dif_round(xv, 1, t, TR, p);
    exchange(xv, S, 1, 2, t);
    dif_round(xv, 2, t, TR, p);
#pragma unroll
    for (int k = 0; k < 16; ++k) xu[k] = mont(xu[k], xv[k], p, pinv);   // in [0, p), carries R^-1, removed in K3
    dit_round(xu, 2, t, TR, p);
    exchange(xu, S, 2, 1, t);
    dit_round(xu, 1, t, TR, p);
    exchange(xu, S, 1, 0, t);
    dit_round(xu, 0, t, TR, p);
#pragma unroll
    for (int k = 0; k < 16; ++k) U[t + 256 * k] = xu[k];                 // in [0, 4p)
}

// ------------------------------------------------- K3: inverse columns --
// grid (4096 / wc3, 1, njobs); LDS: wc3 x n1 residues of one prime at a time.

struct Tri {
    int64_t v, i, c;
};

__device__ __forceinline__ Tri tjoin(Tri a, Tri b) {
    if (b.v > a.v) return b;
    if (a.v > b.v) return a;
    return Tri{a.v, a.i < b.i ? a.i : b.i, a.c + b.c};
}

__global__ void __launch_bounds__(1024) k_ntt_cols_inv(NttGroup g, const NttJob* jobs) {
    extern __shared__ uint32_t L[];
    const NttJob& J = jobs[blockIdx.z];
    const int n1 = g.n1, ln1 = g.log_n1, wc = g.wc3;
    // wc is a power of two: column and row of an index by mask and shift
    // (an integer division per butterfly would cost more than the butterfly)
    const int lwc = __builtin_ctz((unsigned)wc);
    const int b0 = xcd_block(blockIdx.x, gridDim.x) * wc;
    const int tot = wc * n1;
    const uint32_t nmask = ((uint32_t)n1 << 12) - 1u;
    // the primes one after the other in the same LDS; the first prime's
    // scaled residues wait in registers (at most kNttK3Per per thread)
    uint32_t A0[kNttK3Per];
    for (int pr = 0; pr < g.nprimes; ++pr) {
        const uint32_t p = g.p[pr], p2 = 2 * p;
        const uint2* T = tab_of(g, pr);
        const uint32_t* W = J.res + (size_t)pr * ((size_t)n1 << 12);
        uint32_t* Lp = L;
        if (pr) lds_barrier();            // the previous prime's residues are read
        if (tot >= 1024) {
            // as in the forward columns: thread = column c, rows i = i0 +
            // 2^li m, k1 = K + brev(m); f = R w^-(b K), times w^-b per step
            const int c = threadIdx.x & (wc - 1), i0 = threadIdx.x >> lwc, li = 10 - lwc, lm = ln1 - li;
            const uint32_t b = b0 + c, pinv = g.pinv[pr];
            uint32_t f = twist(g.one_m[pr], T, n1, (0u - b * (brev((uint32_t)i0, li) << lm)) & nmask, p);
            f = f >= p ? f - p : f;                                                    // [0, p): W f < 4p^2
            const uint32_t step = twist(g.one_m[pr], T, n1, (0u - b) & nmask, p);      // R w^-b, [0, 2p)
            // the residues of each 16 steps are loaded together
#pragma unroll 1
            for (int m0 = 0; m0 < (1 << lm); m0 += 16) {
                uint32_t wv[16];
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    if (m0 + k < (1 << lm))
                        wv[k] = W[(size_t)b + ((size_t)(i0 + (int)(brev((uint32_t)(m0 + k), lm) << li)) << 12)];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if (m0 + k < (1 << lm)) {
                        const int i = i0 + (int)(brev((uint32_t)(m0 + k), lm) << li);
                        Lp[c + (i << lwc)] = mont(wv[k], f, p, pinv);
                        f = mont(f, step, p, pinv);
                    }
                }
            }
        } else {
            for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
                const int c = idx & (wc - 1), i = idx >> lwc;
                const uint32_t k1 = brev((uint32_t)i, ln1);
                const uint32_t e = ((uint32_t)(b0 + c) * k1) & nmask;
                Lp[idx] = twist(W[(size_t)b0 + c + ((size_t)i << 12)], T, n1, (0u - e) & nmask, p);
            }
        }
        lds_barrier();
        // decimation in time, h = 1 .. n1/2, two stages per pass (h and 2h
        // on the rows r0 = base + pos, r0 + h, r0 + 2h, r0 + 3h of a 4h
        // group, the butterflies of one stage at a time in the same order),
        // then a last single stage when log2(n1) is odd
        int lh = 0;
        // three stages per pass (h, 2h, 4h on the eight rows base + pos +
        // k h of an 8h group) while at least three remain
        for (; lh + 2 < ln1; lh += 3) {
            const int h = 1 << lh;
            const int s1 = ln1 - 1 - lh;
            // the seven twiddles of a group at position pos: stage h (1), 2h (2), 4h (4)
            auto twiddles = [&](int pos, uint2(&w)[7]) {
                w[0] = T[(n1 - (pos << s1)) & (n1 - 1)];
                w[1] = T[(n1 - (pos << (s1 - 1))) & (n1 - 1)];
                w[2] = T[(n1 - ((pos + h) << (s1 - 1))) & (n1 - 1)];
#pragma unroll
                for (int k = 0; k < 4; ++k) w[3 + k] = T[(n1 - ((pos + k * h) << (s1 - 2))) & (n1 - 1)];
            };
            auto group = [&](int bi, const uint2(&w)[7]) {
                const int c = bi & (wc - 1), q = bi >> lwc;
                const int pos = q & (h - 1);
                uint32_t* x0 = &Lp[(((q >> lh) << (lh + 3)) + pos) * wc + c];
                uint32_t x[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) x[k] = x0[k * h * wc];
#pragma unroll
                for (int k = 0; k < 8; k += 2) dit(x[k], x[k + 1], w[0], p, p2);           // stage h
#pragma unroll
                for (int k = 0; k < 8; k += (k & 1) ? 3 : 1)                               // stage 2h: k = 0, 1, 4, 5
                    dit(x[k], x[k + 2], w[1 + (k & 1)], p, p2);
#pragma unroll
                for (int k = 0; k < 4; ++k) dit(x[k], x[k + 4], w[3 + k], p, p2);          // stage 4h
#pragma unroll
                for (int k = 0; k < 8; ++k) x0[k * h * wc] = x[k];
            };
            if (((int)blockDim.x >> lwc) % h == 0) {
                // every group of this thread has the same position: twiddles once
                uint2 w[7];
                twiddles((int)(threadIdx.x >> lwc) & (h - 1), w);
                for (int bi = threadIdx.x; bi < tot / 8; bi += blockDim.x) group(bi, w);
            } else {
                for (int bi = threadIdx.x; bi < tot / 8; bi += blockDim.x) {
                    uint2 w[7];
                    twiddles((bi >> lwc) & (h - 1), w);
                    group(bi, w);
                }
            }
            lds_barrier();
        }
        if (lh + 1 < ln1) {
            const int h = 1 << lh;
            const int s1 = ln1 - 1 - lh;         // stage h; stage 2h uses s1 - 1
            for (int bi = threadIdx.x; bi < tot / 4; bi += blockDim.x) {
                const int c = bi & (wc - 1), q = bi >> lwc;
                const int pos = q & (h - 1);
                const int r0 = ((q >> lh) << (lh + 2)) + pos;
                uint32_t* x0 = &Lp[r0 * wc + c];
                uint32_t* x1 = x0 + h * wc;
                uint32_t* x2 = x1 + h * wc;
                uint32_t* x3 = x2 + h * wc;
                const uint2 w1 = T[(n1 - (pos << s1)) & (n1 - 1)];
                uint32_t a0 = *x0, a1 = *x1, a2 = *x2, a3 = *x3;
                dit(a0, a1, w1, p, p2);                                      // stage h
                dit(a2, a3, w1, p, p2);
                dit(a0, a2, T[(n1 - (pos << (s1 - 1))) & (n1 - 1)], p, p2);  // stage 2h
                dit(a1, a3, T[(n1 - ((pos + h) << (s1 - 1))) & (n1 - 1)], p, p2);
                *x0 = a0;
                *x1 = a1;
                *x2 = a2;
                *x3 = a3;
            }
            lds_barrier();
            lh += 2;
        }
        if (lh == ln1 - 1) {
            const int h = 1 << lh;
            for (int bi = threadIdx.x; bi < tot / 2; bi += blockDim.x) {
                const int c = bi & (wc - 1), pos = bi >> lwc;          // one group: e = pos
                uint32_t a = Lp[pos * wc + c], b = Lp[(pos + h) * wc + c];
                dit(a, b, T[(n1 - pos) & (n1 - 1)], p, p2);
                Lp[pos * wc + c] = a;
                Lp[(pos + h) * wc + c] = b;
            }
            lds_barrier();
        }
        if (pr == 0 && g.nprimes == 2) {
#pragma unroll
            for (int m = 0; m < kNttK3Per; ++m) {
                const int idx = threadIdx.x + m * 1024;
                if (idx < tot) A0[m] = mont(L[idx], g.scale_m[0], p, g.pinv[0]);   // L < 4p: [0, p1)
            }
        }
    }
    // scale, CRT, outputs
    Tri tr{INT64_MIN, INT64_MAX, 0};
#pragma unroll
    for (int m = 0; m < kNttK3Per; ++m) {
        const int idx = threadIdx.x + m * 1024;
        const int c = idx & (wc - 1), i = idx >> lwc;
        const int64_t j = b0 + c + ((int64_t)i << 12);
        if (idx >= tot || j < J.jlo || j > J.jhi) continue;
        int64_t val;
        if (g.nprimes == 1) {
            const uint32_t a1 = mont(L[idx], g.scale_m[0], g.p[0], g.pinv[0]);     // L < 4p: a1 in [0, p1)
            val = a1 > (g.p[0] - 1) / 2 ? (int64_t)a1 - (int64_t)g.p[0] : (int64_t)a1;
        } else {
            const uint32_t a1 = A0[m];
            const uint32_t a2 = mont(L[idx], g.scale_m[1], g.p[1], g.pinv[1]);
            const uint32_t a1r = a1 >= g.p[1] ? a1 - g.p[1] : a1;
            const uint32_t d = subm(a2, a1r, g.p[1]);
            const uint32_t tq = mont(d, g.crt_m, g.p[1], g.pinv[1]);       // (a2 - a1) p1^-1 mod p2
            const uint64_t x = (uint64_t)a1 + (uint64_t)g.p[0] * tq;        // in [0, p1 p2)
            const uint64_t M = (uint64_t)g.p[0] * g.p[1];
            val = x > (M - 1) / 2 ? (int64_t)(x - M) : (int64_t)x;
        }
        const int64_t ri = j - (J.nu - 1) - J.lag_lo;
        if (J.r) {
            if (J.r_dtype == TDE_I32) static_cast<int32_t*>(J.r)[ri] = (int32_t)val;
            else static_cast<int64_t*>(J.r)[ri] = val;
        }
        tr = tjoin(tr, Tri{val, ri, 1});
    }
    if (!J.parts) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Tri u{__shfl_xor(tr.v, o, 64), __shfl_xor(tr.i, o, 64), __shfl_xor(tr.c, o, 64)};
        tr = tjoin(tr, u);
    }
    __shared__ Tri sh[16];
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = tr;
    __syncthreads();
    if (threadIdx.x == 0) {
        Tri a = sh[0];
        for (int k = 1; k < nw; ++k) a = tjoin(a, sh[k]);
        J.parts[blockIdx.x] = ArgPart{a.v, a.i, a.c};
    }
}

uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = (unsigned __int128)r * a % p;
        a = (unsigned __int128)a * a % p;
        e >>= 1;
    }
    return r;
}

uint32_t to_mont(uint64_t x, uint32_t p) { return (uint32_t)(((unsigned __int128)(x % p) << 32) % p); }

}  // namespace

// ---------------------------------------------------------------- host --

bool ntt_plan(int64_t nu, int64_t nv, int kuv, int64_t lag_lo, int64_t lag_hi, NttPlan& P) {
    // positions j = tau + nu - 1 of the lags inside the support
    const int64_t lo = std::max<int64_t>(lag_lo, -(nu - 1));
    const int64_t hi = std::min<int64_t>(lag_hi, nv - 1);
    P.jlo = lo + nu - 1;
    P.jhi = hi + nu - 1;
    int64_t need = 1;
    if (P.jlo <= P.jhi) need = std::max<int64_t>(P.jhi + 1, nu + nv - 1 - P.jlo);
    int L = kNttMinLog;
    while (L < kNttMaxLog && ((int64_t)1 << L) < need) ++L;
    if (((int64_t)1 << L) < need) return false;
    P.log_n = L;
    // one prime while every |r| < p1 / 2
    const int64_t ov = std::min(nu, nv);
    P.nprimes = ((__int128)ov * kuv < (__int128)(kP[0] / 2)) ? 1 : 2;
    const int n1 = 1 << (L - 12);
    P.wc3 = std::min(kNttC1, (int)(32768 / n1));      // one prime at a time in LDS
    P.ntiles = kNttRow / P.wc3;
    return true;
}

// (w, quotient) pairs: two words per entry
size_t ntt_tab_words(const NttPlan& P) { return (size_t)P.nprimes * 2 * ((1u << (P.log_n - 12)) + 2 * kNttRow); }

size_t ntt_res_bytes(const NttPlan& P) { return (size_t)2 * P.nprimes * ((size_t)4 << P.log_n); }

NttGroup ntt_group(const NttPlan& P, uint32_t* tab) {
    NttGroup g{};
    g.tab = tab;
    g.log_n = P.log_n;
    g.log_n1 = P.log_n - 12;
    g.n1 = 1 << g.log_n1;
    g.nprimes = P.nprimes;
    g.wc3 = P.wc3;
    const uint64_t n = (uint64_t)1 << P.log_n;
    for (int pr = 0; pr < 2; ++pr) {
        const uint32_t p = kP[pr];
        uint32_t inv = 1;                                  // p^-1 mod 2^32 by Newton steps
        for (int k = 0; k < 5; ++k) inv *= 2u - p * inv;
        g.p[pr] = p;
        g.pinv[pr] = inv;
        g.one_m[pr] = to_mont(1, p);
        g.root_m[pr] = to_mont(powmod(kG[pr], (p - 1) / n, p), p);
        // n^-1 R, in Montgomery form: removes the R^-1 of the pointwise product
        const uint64_t ninv = powmod(n, p - 2, p);
        g.scale_m[pr] = to_mont((unsigned __int128)ninv * (((uint64_t)1 << 32) % p) % p, p);
    }
    g.crt_m = to_mont(powmod(kP[0] % kP[1], kP[1] - 2, kP[1]), kP[1]);
    return g;
}

int launch_ntt(const NttGroup& g, const NttJob* jobs_dev, int njobs, hipStream_t s) {
    if (njobs == 0) return TDE_OK;
    const int per = (g.n1 + 2 * kNttRow) * g.nprimes;
    hipLaunchKernelGGL(k_ntt_tables, dim3(ceil_div(per, 256)), dim3(256), 0, s, g);
    TDE_HIP_CHECK(hipGetLastError());
    static bool attr = false;
    if (!attr) {
        TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_ntt_cols_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          kNttC1 * 2048 * 4));
        TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_ntt_cols_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          32768 * 4));
        attr = true;
    }
    hipLaunchKernelGGL(k_ntt_cols_fwd, dim3(kNttRow / kNttC1, 2, njobs), dim3(1024),
                       kNttC1 * g.n1 * 4, s, g, jobs_dev);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_ntt_rows, dim3(g.n1, g.nprimes, njobs), dim3(256), 0, s, g, jobs_dev);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_ntt_cols_inv, dim3(kNttRow / g.wc3, 1, njobs), dim3(1024), g.wc3 * g.n1 * 4, s, g,
                       jobs_dev);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
