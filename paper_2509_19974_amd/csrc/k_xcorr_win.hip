// Algorithm 1, correlation step restricted to proposed lag windows: the exact integer
// correlation r[tau] = sum_m u[m] v[m + tau] (Eq. (1)) over windows of 256
// consecutive lags, with each window's (max, smallest lag, count) triple as
// the only output. Two kernels:
//
// k_xcorr_win_fp (codes up to 3 / 7: FP4 / FP6 operands of
// v_mfma_scale_f32_32x32x64_f8f6f4, fp32 accumulation of integers, exact
// while a wave's partial sum stays below 2^24): one workgroup per pair, all
// of its windows (at most 8) in one 32-row tile. Row i = 8 g + w is group g
// of window w, with lag offset f(g) = 32 (g mod 2) + 128 floor(g / 2), i.e.
// 0, 32, 128, 160; column j, column block b in {0, 1}:
//     tau = T0_w + f(g) + 64 b + j
//     A[i][k]   = v[q + T0_w + f(g) + k]       k in [0, 64)
//     B_b[k][j] = u[q + k - j - 64 b]          the same for every window
// so C_b[i][j] collects u[m] v[m + tau] for m = q + k - j - 64 b, and the
// offsets {f(g) + 64 b + j} cover the window's 256 lags once. B_0 feeds both
// matrix instructions of all 8 windows, and B_1 of a step is B_0 of the step
// before (q - 64) in the same lane: each step reads one 32-code u piece per
// lane.
//
// k_xcorr_win (int8 operands, v_mfma_i32_16x16x64_i8, int32 accumulation):
// one workgroup per 4 windows, for int8 codes or more than 8 windows. Row
// i = 4 w + r is lag offset 16 r of window w, column j, column block b < 4:
//     tau = T0_w + 16 r + 64 b + j
//     A[i][k]   = v[q + T0_w + 16 r + k]   (16-byte row pieces)
//     B_b[k][j] = u[q + k - j - 64 b]      (Hankel in (k, j), the same for every window)
//     C_b[i][j] += sum_k A[i][k] B_b[k][j] collects u[m] v[m + tau], m = q + k - j - 64 b
// so the offsets 16 r + 64 b + j cover a window's 256 lags once, and B_b at
// step q is B_0 at step q - 64 b in the same lane: a step reads one A piece
// and one B_0 piece per lane for 4 matrix instructions.
//
// In both, for each column the steps q = Qa, Qa + 64, ... cover a contiguous
// m range, so Qa <= first m and Qb >= last m + j + 64 b make every sum
// complete; samples outside the signals are staged as 0 (finite
// support, Section 2.2). The 4 waves of a workgroup take a quarter of the
// steps each, staging their own chunk of u and v in LDS; partial tiles meet
// in LDS in int64. Each wave's partial covers at most a quarter of the m
// range, which the host keeps below 2^24 / (Ku Kv) values for the FP kernel
// and (2^31 - 1) / (Ku Kv) for the int8 one.
#include "tde_internal.h"

namespace tde {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kW8Steps = 32;                    // steps of 64 m per staged chunk
constexpr int kW8CM = 64 * kW8Steps;            // m per chunk
// v bytes of a window region: rows reach 16 r + k < 112 past the chunk's last
// step; the 64 bytes of padding (a region is 64 mod 128 bytes) put the
// 16-byte row pieces that one LDS pass serves (8 lanes: 2 windows x 4 rows)
// on distinct banks
constexpr int kW8V = kW8CM + 128 + 64;
constexpr int kW8U = kW8CM + 288;               // u bytes from q0 - 208: B_0 pieces end by q + 64, plus one dword
constexpr int kW8Wave = 4 * kW8V + kW8U;
static_assert(kW8V % 128 == 64 && kW8U % 16 == 0, "region layout");
static_assert(4 * kW8Wave >= 4 * 256 * 8, "the reduction area must fit");

__device__ __forceinline__ uint4 ld16(const int8_t* base, int64_t n, int64_t gi) {
    const int8_t* p = base + gi;
    if (gi >= 0 && gi + 16 <= n && ((((uintptr_t)p) & 15) == 0)) return gload16(p);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (gi + 16 > 0 && gi < n) {
        for (int e = 0; e < 16; ++e) {
            const int64_t idx = gi + e;
            const uint32_t byte = (idx >= 0 && idx < n) ? gload_u8(base + idx) : 0u;
            w[e >> 2] |= byte << (8 * (e & 3));
        }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

struct Tri {
    int64_t v, i, c;
};

__device__ __forceinline__ Tri tjoin(Tri a, Tri b) {
    if (b.v > a.v) return b;
    if (a.v > b.v) return a;
    return Tri{a.v, a.i < b.i ? a.i : b.i, a.c + b.c};
}

}  // namespace

// grid (npairs * ceil(topk / 4)): workgroup -> (pair, group of 4 windows).
// Pairs whose margin is below theta (full-range fallback) are skipped.
__global__ void __launch_bounds__(256) k_xcorr_win(const XItem* items, const int32_t* top, const float* margin,
                                                   float theta, int topk, int nb, ArgPart* parts) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[4 * kW8Wave];
    __shared__ int64_t s_t0[4];
    const int ngrp = (topk + 3) / 4;
    const int pair = blockIdx.x / ngrp, grp = blockIdx.x % ngrp;
    if (!(margin[pair] >= theta)) return;          // fallback pair (also NaN)
    const XItem& it = items[pair];
    if (it.win_w != 0) return;                     // windows on the FP kernel
    // descriptor fields in registers (the LDS stores below go through
    // generic pointers, after which fields read through `it` are reloaded)
    const int8_t* up = it.p.u;
    const int8_t* vp = it.p.v;
    const int64_t nu = it.p.nu, nv = it.p.nv, lag_lo = it.p.lag_lo, lag_hi = it.p.lag_hi;
    const int nw = topk - 4 * grp < 4 ? topk - 4 * grp : 4;     // live windows of the group
    if (threadIdx.x < 4)
        s_t0[threadIdx.x] =
            (int)threadIdx.x < nw ? (int64_t)(top[(int64_t)pair * topk + 4 * grp + threadIdx.x] - nb / 2) * 256 : 0;
    __syncthreads();
    // the union of the live windows' m ranges (zero outside the signals)
    int64_t m_lo = INT64_MAX, m_hi = INT64_MIN;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < nw) {
            const int64_t t0 = s_t0[w];
            const int64_t lo = t0 + 255 < 0 ? -(t0 + 255) : 0;
            const int64_t hi = nu < nv - t0 ? nu : nv - t0;
            if (hi > lo) {
                m_lo = lo < m_lo ? lo : m_lo;
                m_hi = hi > m_hi ? hi : m_hi;
            }
        }
    }
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform in the wave
    v4i acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = v4i{0, 0, 0, 0};
    if (m_hi > m_lo) {
        // block b covers m in [Qa - j - 64 b, Qb - j - 64 b): Qa <= m_lo and
        // Qb >= m_hi + 15 + 192 include every nonzero term once
        const int64_t Qa = floor_div(m_lo, 64) * 64;
        const int64_t Qb = ceil_div(m_hi + 207, 64) * 64;
        // whole groups of 4 steps per wave (the history slots rotate by 4);
        // steps past Qb meet only zero samples
        const int64_t nsteps = (Qb - Qa) / 64;
        const int64_t per = round_up(ceil_div(nsteps, 4), 4);
        const int64_t sa = wv * per, sb = sa + per;
        uint8_t* vb = lds + wv * kW8Wave;
        uint8_t* ub = vb + 4 * kW8V;
        const int i = lane & 15, kq = lane >> 4;
        const int w = i >> 2, r = i & 3;
        // regions of windows past the live ones read zeros: cleared once
        // here and never staged (the wave's own area; its LDS accesses take
        // effect in order)
        for (int ww = nw; ww < 4; ++ww)
            for (int o = 16 * lane; o < kW8V; o += 1024)
                *reinterpret_cast<uint4*>(vb + ww * kW8V + o) = make_uint4(0u, 0u, 0u, 0u);
        // A row i = 4 w + r: window w's region, lag offset 16 r, k bytes 16 kq ..
        const uint8_t* arow = vb + w * kW8V + 16 * r + 16 * kq;
        // B_0 piece of this lane (column j = i, k bytes 16 kq ..) at step s of
        // a chunk: u[q + 16 kq - j ..], at byte 64 s + 208 + 16 kq - j of the
        // u region (which starts at q0 - 208)
        const int b_off = 208 + 16 * kq - i;
        const uint32_t* bw0 = reinterpret_cast<const uint32_t*>(ub + (b_off & ~3));
        const uint32_t sh8 = (uint32_t)(b_off & 3);
        auto piece = [&](int s) {                   // B_0 of step s (s >= -3)
            const uint32_t* bw = bw0 + 16 * s;
            uint32_t d[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) d[k] = bw[k];
            v4i b;
#pragma unroll
            for (int k = 0; k < 4; ++k) b[k] = (int)__builtin_amdgcn_alignbyte(d[k + 1], d[k], sh8);
            return b;
        };
        // slot t holds B_0 of the step = t (mod 4); block b at step s takes
        // slot (s - b) mod 4, B_0 of step s - b
        v4i hb[4];
        // staging of a chunk: v[q0 + T0_w, + kW8V) of the live windows and
        // u[q0 - 208, + kW8U), 16-byte units; the next chunk's units are
        // loaded into registers while the current chunk runs
        constexpr int VU = kW8V / 16, UU = kW8U / 16;
        constexpr int PER_LANE = (4 * VU + UU + 63) / 64;
        uint4 reg[PER_LANE];
        auto load = [&](int64_t q0) {
#pragma unroll
            for (int k = 0; k < PER_LANE; ++k) {
                const int unit = lane + 64 * k;
                if (unit < 4 * VU) {
                    const int ww = unit / VU, uu = unit - ww * VU;
                    if (ww < nw) reg[k] = ld16(vp, nv, q0 + s_t0[ww] + 16 * uu);
                } else if (unit < 4 * VU + UU) {
                    reg[k] = ld16(up, nu, q0 - 208 + 16 * (unit - 4 * VU));
                }
            }
        };
        auto store = [&]() {
#pragma unroll
            for (int k = 0; k < PER_LANE; ++k) {
                const int unit = lane + 64 * k;
                if (unit < 4 * VU) {
                    const int ww = unit / VU, uu = unit - ww * VU;
                    if (ww < nw) *reinterpret_cast<uint4*>(vb + ww * kW8V + 16 * uu) = reg[k];
                } else if (unit < 4 * VU + UU) {
                    *reinterpret_cast<uint4*>(ub + 16 * (unit - 4 * VU)) = reg[k];
                }
            }
        };
        load(Qa + 64 * sa);
        for (int64_t s0 = sa; s0 < sb; s0 += kW8Steps) {
            const int ns = (int)(sb - s0 < kW8Steps ? sb - s0 : kW8Steps);     // a multiple of 4
            store();                                // this wave's reads of the last chunk are done (in order)
            if (s0 + kW8Steps < sb) load(Qa + 64 * (s0 + kW8Steps));
            if (s0 == sa) {
                hb[3] = piece(-1);
                hb[2] = piece(-2);
                hb[1] = piece(-3);
            }
            for (int s = 0; s < ns; s += 4) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint4 av = *reinterpret_cast<const uint4*>(arow + 64 * (s + t));
                    const v4i a = {(int)av.x, (int)av.y, (int)av.z, (int)av.w};
                    hb[t] = piece(s + t);
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        acc[b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, hb[(t - b) & 3], acc[b], 0, 0, 0);
                }
            }
        }
    }
    // the waves' partials meet in LDS (int64): red[w][lag offset in the window];
    // output layout: lane -> column j = lane % 16, rows 4 (lane / 16) + e, so
    // a lane's rows all belong to window lane / 16
    __syncthreads();
    long long* red = reinterpret_cast<long long*>(lds);
    for (int k = threadIdx.x; k < 4 * 256; k += 256) red[k] = 0;
    __syncthreads();
    {
        const int j = lane & 15, gq = lane >> 4;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (acc[b][e])
                    atomicAdd((unsigned long long*)&red[gq * 256 + 16 * e + 64 * b + j],
                              (unsigned long long)(long long)acc[b][e]);
    }
    __syncthreads();
    // wave wv: the triple of window wv of the group
    if (wv < nw) {
        Tri t{INT64_MIN, INT64_MAX, 0};
        const int64_t base = s_t0[wv] - lag_lo;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int k = lane + 64 * rr;
            const int64_t idx = base + k;
            if (idx >= 0 && idx <= lag_hi - lag_lo) t = tjoin(t, Tri{(int64_t)red[wv * 256 + k], idx, 1});
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            Tri u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
            t = tjoin(t, u);
        }
        if (lane == 0) parts[(int64_t)pair * topk + 4 * grp + wv] = ArgPart{t.v, t.i, t.c};
    }
}

// ------------------------------------------------------------ FP operands --
template <int W>
struct WinFp {
    static constexpr int KS = 64;                 // m per matrix step
    static constexpr int CQ = 16;                 // steps per staged chunk
    static constexpr int CM = KS * CQ;            // m per chunk
    static constexpr int VWIN = CM + 192;         // v codes of a window region: rows reach f(g) + k < 224
    static constexpr int UWIN = CM + 144;         // u codes from q0 - 128: B_0 pieces end by q + 64, plus one dword
    // padded bytes of a window region: A rows are read as 8-byte (FP6) or
    // 16-byte (FP4) pieces, so regions and wave areas keep 16-byte alignment;
    // with rows i = 8 g + w, 32 (FP6) or 16 (FP4) bytes of padding put the
    // pieces that 16 lanes read together (8 or 4 bytes each) on distinct
    // banks of a 32-bank LDS
    static constexpr int VB = VWIN * W / 8 + (W == 6 ? 32 : 16);
    static constexpr int UB = UWIN * W / 8;
    static constexpr int WAVE_LDS = (8 * VB + UB + 15) / 16 * 16;
    static constexpr int VUNITS = VWIN / 16, UUNITS = UWIN / 16;
    static constexpr int UNITS = 8 * VUNITS + UUNITS;
    static constexpr int PER_LANE = (UNITS + 63) / 64;
    static_assert(VWIN % 16 == 0 && UWIN % 16 == 0, "regions are whole 16-code units");
    static_assert(VB % 16 == 0, "16-byte aligned window regions");
    static_assert(4 * WAVE_LDS >= 8 * 256 * 8, "the reduction area must fit");
};

// grid npairs: workgroup -> pair. Pairs below the margin threshold (full-range
// fallback) and pairs whose windows run on the int8 kernel are skipped.
template <int W>
__global__ void __launch_bounds__(256) k_xcorr_win_fp(const XItem* items, const int32_t* top, const float* margin,
                                                      float theta, int topk, int nb, ArgPart* parts) {
    using C = WinFp<W>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[4 * C::WAVE_LDS];
    __shared__ int64_t s_t0[8];
    const int pair = blockIdx.x;
    if (!(margin[pair] >= theta)) return;          // fallback pair (also NaN)
    const XItem& it = items[pair];
    if (it.win_w != W) return;
    // descriptor fields in registers (LDS stores below go through generic
    // pointers, after which fields read through `it` would be reloaded)
    const uint32_t* upk = it.p.upk;
    const uint32_t* vpk = it.p.vpk;
    const int64_t nu = it.p.nu, nv = it.p.nv, lag_lo = it.p.lag_lo, lag_hi = it.p.lag_hi;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform in the wave
    // the windows' first lags (an LDS table: the staging loop indexes it by
    // a computed window); the union of their m ranges
    if (threadIdx.x < 8)
        s_t0[threadIdx.x] = (int)threadIdx.x < topk ? (int64_t)(top[(int64_t)pair * topk + threadIdx.x] - nb / 2) * 256
                                                    : 0;
    __syncthreads();
    int64_t m_lo = INT64_MAX, m_hi = INT64_MIN;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        if (w < topk) {
            const int64_t t0 = s_t0[w];
            const int64_t lo = t0 + 255 < 0 ? -(t0 + 255) : 0;
            const int64_t hi = nu < nv - t0 ? nu : nv - t0;
            if (hi > lo) {
                m_lo = lo < m_lo ? lo : m_lo;
                m_hi = hi > m_hi ? hi : m_hi;
            }
        }
    }
    v16f acc0, acc1;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc0[e] = acc1[e] = 0.f;
    if (m_hi > m_lo) {
        // block b covers m in [Qa - j - 64 b, Qb - j - 64 b): Qa <= m_lo and
        // Qb >= m_hi + 31 + 64 include every nonzero term once
        const int64_t Qa = floor_div(m_lo, 64) * 64;
        const int64_t Qb = ceil_div(m_hi + 95, 64) * 64;
        // whole chunks per wave: steps past Qb meet only zero samples (each
        // window's m range ends by Qb - 95), so they add nothing
        const int64_t nsteps = (Qb - Qa) / 64;
        const int64_t per = round_up(ceil_div(nsteps, 4), C::CQ);
        const int64_t sa = wv * per, sb = sa + per;
        uint8_t* vb = lds + wv * C::WAVE_LDS;
        uint8_t* ub = vb + 8 * C::VB;
        const int i = lane & 31, kh = lane >> 5;
        const int w = i & 7, g = i >> 3;
        // A row of this lane: window w's region, group g, k half kh
        const int fg = 32 * (g & 1) + 128 * (g >> 1);
        const uint8_t* arow = vb + w * C::VB + ((fg + 32 * kh) * W) / 8;
        // B_0 piece of this lane (column j = i, k half kh) at step s of a
        // chunk: 32 codes from code 64 s + 128 + 32 kh - j of the u region
        const int brel = 128 + 32 * kh - i;
        const uint32_t* ubw = reinterpret_cast<const uint32_t*>(ub) + ((W * brel) >> 5);
        const uint32_t bsh = (uint32_t)((W * brel) & 31);
        Packed16<W> reg[C::PER_LANE];
        auto load = [&](int64_t q0) {
#pragma unroll
            for (int k = 0; k < C::PER_LANE; ++k) {
                const int unit = lane + 64 * k;
                if (unit < 8 * C::VUNITS) {
                    const int ww = unit / C::VUNITS, uu = unit - ww * C::VUNITS;
                    if (ww < topk) reg[k] = load_unit<W>(vpk, nv, (q0 + s_t0[ww]) / 16 + uu);
                } else if (unit < C::UNITS) {
                    reg[k] = load_unit<W>(upk, nu, (q0 - 128) / 16 + (unit - 8 * C::VUNITS));
                }
            }
        };
        auto store = [&]() {
#pragma unroll
            for (int k = 0; k < C::PER_LANE; ++k) {
                const int unit = lane + 64 * k;
                uint8_t* dst = nullptr;
                if (unit < 8 * C::VUNITS) {
                    const int ww = unit / C::VUNITS, uu = unit - ww * C::VUNITS;
                    if (ww < topk) dst = vb + ww * C::VB + 2 * W * uu;
                } else if (unit < C::UNITS) {
                    dst = ub + 2 * W * (unit - 8 * C::VUNITS);
                }
                if (dst) {
                    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
                    for (int e = 0; e < W / 2; ++e) d[e] = reg[k].d[e];
                }
            }
        };
        constexpr int ASTEP = C::KS * W / 8;       // bytes per step along a row
        // rows of windows past topk read zeros: their regions are cleared
        // once here and never staged (the wave's own area; its LDS accesses
        // take effect in order)
        for (int ww = topk; ww < 8; ++ww)
            for (int o = 4 * lane; o < C::VB; o += 256) *reinterpret_cast<uint32_t*>(vb + ww * C::VB + o) = 0u;
        load(Qa + 64 * sa);
        v8i b1;                                     // B_0 of the previous step
        for (int64_t s0 = sa; s0 < sb; s0 += C::CQ) {
            store();                                // this wave's reads of the last chunk are done (in order)
            if (s0 + C::CQ < sb) load(Qa + 64 * (s0 + C::CQ));
            if (s0 == sa) b1 = split_piece<W>(read_piece<W>(ubw - 2 * W), bsh);   // step sa - 1
            // fragments of step s + 2 are read while the matrix
            // instructions of step s run
            v8i a = read_a_fp<W>(arow), a_nx = read_a_fp<W>(arow + ASTEP);
            BPiece<W> raw = read_piece<W>(ubw), raw_nx = read_piece<W>(ubw + 2 * W);
#pragma unroll
            for (int s = 0; s < C::CQ; ++s) {
                const v8i b0 = split_piece<W>(raw, bsh);
                const v8i a_cur = a;
                a = a_nx;
                raw = raw_nx;
                if (s + 2 < C::CQ) {
                    a_nx = read_a_fp<W>(arow + ASTEP * (s + 2));
                    raw_nx = read_piece<W>(ubw + 2 * W * (s + 2));
                }
                __builtin_amdgcn_sched_barrier(0);
                acc1 = mfma_fp<W>(a_cur, b1, acc1);
                acc0 = mfma_fp<W>(a_cur, b0, acc0);
                __builtin_amdgcn_sched_barrier(0);
                b1 = b0;
            }
        }
    }
    // the waves' partials meet in LDS (int64): red[w][lag offset in the window]
    __syncthreads();
    long long* red = reinterpret_cast<long long*>(lds);
    for (int k = threadIdx.x; k < 8 * 256; k += 256) red[k] = 0;
    __syncthreads();
    {
        const int j = lane & 31, gq = lane >> 5;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = 8 * (e >> 2) + 4 * gq + (e & 3);
            const int w = i & 7, g = i >> 3;
            const int o = w * 256 + 32 * (g & 1) + 128 * (g >> 1) + j;
            const int v0 = (int)acc0[e], v1 = (int)acc1[e];
            if (v0) atomicAdd((unsigned long long*)&red[o], (unsigned long long)(long long)v0);
            if (v1) atomicAdd((unsigned long long*)&red[o + 64], (unsigned long long)(long long)v1);
        }
    }
    __syncthreads();
    // wave wv: the triples of windows 2 wv and 2 wv + 1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int w = 2 * wv + h;
        Tri t{INT64_MIN, INT64_MAX, 0};
        if (w < topk) {
            const int64_t base = s_t0[w] - lag_lo;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = lane + 64 * r;
                const int64_t idx = base + k;
                if (idx >= 0 && idx <= lag_hi - lag_lo) t = tjoin(t, Tri{(int64_t)red[w * 256 + k], idx, 1});
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            Tri u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
            t = tjoin(t, u);
        }
        if (lane == 0 && w < topk) parts[(int64_t)pair * topk + w] = ArgPart{t.v, t.i, t.c};
    }
}

int launch_xcorr_win(const XItem* items_dev, int npairs, const int32_t* top, const float* margin, float theta,
                     int topk, int nb, ArgPart* parts, hipStream_t s, int formats) {
    if (npairs == 0) return TDE_OK;
    if (formats & 1)
        hipLaunchKernelGGL(k_xcorr_win, dim3(npairs * ((topk + 3) / 4)), dim3(256), 0, s, items_dev, top, margin, theta,
                           topk, nb, parts);
    if (formats & 2)
        hipLaunchKernelGGL(k_xcorr_win_fp<6>, dim3(npairs), dim3(256), 0, s, items_dev, top, margin, theta, topk, nb,
                           parts);
    if (formats & 4)
        hipLaunchKernelGGL(k_xcorr_win_fp<4>, dim3(npairs), dim3(256), 0, s, items_dev, top, margin, theta, topk, nb,
                           parts);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
