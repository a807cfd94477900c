// Algorithm 1, line 3 (Eq. (1) on integer codes), exact, on the int8 matrix
// cores of gfx950 (v_mfma_i32_32x32x32_i8, int32 accumulation).
//
// The correlation r[tau] = sum_m u[m] v[m + tau] is a product of a Hankel
// and a Toeplitz matrix. One wave owns 1024*MB consecutive lags
//     tau = Tw + c + S*i,   c = j + 32 b in [0, S),  S = 32 MB,  i, j in [0, 32)
// held in MB accumulator tiles C_b[i][j] (rows i: coarse lag, columns j: fine
// lag, so the 32 lanes of a tile row hold 32 consecutive lags). The k loop
// walks m in steps of 32:
//     A[i][k]   = v[q + Tw + S i + k]        (rows S bytes apart, 16-byte aligned)
//     B_b[k][j] = u[q + k - j - 32 b]        (Hankel in (k, j))
//     C_b      += A x B_b
// so C_b[i][j] collects u[m] v[m + tau] for m = q + k - j - 32 b. The Hankel
// structure gives B_b(q) = B_0(q - 32 b): each step loads one new B fragment
// and one A fragment for MB matrix instructions; the other MB-1 B fragments
// are the previous steps' B_0, kept in registers.
//
// Windows of v and u for a chunk of 64 steps are staged in LDS (double
// buffered) by the whole workgroup; out-of-range samples are staged as 0,
// which is the finite-length (zero outside the support) convention of
// Section 2.2. A rows are read with 16-byte LDS reads through an XOR swizzle
// (rows S bytes apart would otherwise fall into one bank group); B rows start
// at arbitrary byte offsets and are assembled from 5 aligned dwords with
// v_alignbyte.
//
// Partial sums per work item cover at most floor((2^31-1)/(Ku Kv)) values of
// m, so no int32 accumulator can overflow (coefficient bound of Section 3.2);
// items add their partials to r with integer atomics, which are exact and
// order-independent.
#include "tde_internal.h"

namespace tde {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

template <int MB>
struct MCfg {
    static constexpr int S = 32 * MB;          // coarse lag stride, A row stride
    static constexpr int LS = MB == 1 ? 5 : MB == 2 ? 6 : MB == 4 ? 7 : 8;
    static constexpr int WAVES = 4;
    static constexpr int TLW = 32 * S;         // lags per wave
    static constexpr int TL = WAVES * TLW;     // lags per workgroup
    static constexpr int CQ = 64;              // k steps per staged chunk
    static constexpr int CM = 32 * CQ;         // m per chunk
    static constexpr int VW = TL + CM;         // staged v bytes
    static constexpr int UOFF = 32 * MB;       // u window starts UOFF before the chunk
    static constexpr int UW = CM + UOFF + 64;  // staged u bytes (multiple of 16)
    static constexpr int BUF = VW + UW;
    static constexpr int LDS = 2 * BUF;
    static constexpr int VUNITS = VW / 16;
    static constexpr int UUNITS = UW / 16;
    static constexpr int PER_THREAD = (VUNITS + UUNITS + 255) / 256;
};

// XOR swizzle of 16-byte chunks inside 128-byte rows, keyed by the A row.
template <int LS>
__device__ __forceinline__ int swz(int t) {
    return t ^ (((t >> LS) & 7) << 4);
}

__device__ __forceinline__ uint4 load16_guarded(const int8_t* base, int64_t n, int64_t gi) {
    const int8_t* p = base + gi;
    if (gi >= 0 && gi + 16 <= n && ((((uintptr_t)p) & 15) == 0)) {
        return *reinterpret_cast<const uint4*>(p);
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (gi + 16 > 0 && gi < n) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int64_t idx = gi + e;
            uint32_t byte = (idx >= 0 && idx < n) ? (uint32_t)(uint8_t)base[idx] : 0u;
            w[e >> 2] |= byte << (8 * (e & 3));
        }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <int MB>
struct Stager {
    using C = MCfg<MB>;
    uint4 reg[C::PER_THREAD];

    __device__ __forceinline__ void load(const XPair& p, int64_t T0, int64_t qc) {
        const int64_t gv0 = qc + T0;
        const int64_t gu0 = qc - C::UOFF;
#pragma unroll
        for (int k = 0; k < C::PER_THREAD; ++k) {
            int unit = threadIdx.x + 256 * k;
            if (unit < C::VUNITS) {
                reg[k] = load16_guarded(p.v, p.nv, gv0 + 16 * (int64_t)unit);
            } else if (unit < C::VUNITS + C::UUNITS) {
                reg[k] = load16_guarded(p.u, p.nu, gu0 + 16 * (int64_t)(unit - C::VUNITS));
            }
        }
    }
    __device__ __forceinline__ void store(uint8_t* buf) {
#pragma unroll
        for (int k = 0; k < C::PER_THREAD; ++k) {
            int unit = threadIdx.x + 256 * k;
            if (unit < C::VUNITS) {
                *reinterpret_cast<uint4*>(buf + swz<C::LS>(16 * unit)) = reg[k];
            } else if (unit < C::VUNITS + C::UUNITS) {
                *reinterpret_cast<uint4*>(buf + C::VW + 16 * (unit - C::VUNITS)) = reg[k];
            }
        }
    }
};

// 16 bytes of the staged u window starting at byte t (any alignment).
__device__ __forceinline__ v4i read_b(const uint8_t* ub, int t) {
    const uint32_t* d = reinterpret_cast<const uint32_t*>(ub) + (t >> 2);
    const uint32_t sh = (uint32_t)(t & 3);
    uint32_t d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3], d4 = d[4];
    v4i r;
    r[0] = (int)__builtin_amdgcn_alignbyte(d1, d0, sh);
    r[1] = (int)__builtin_amdgcn_alignbyte(d2, d1, sh);
    r[2] = (int)__builtin_amdgcn_alignbyte(d3, d2, sh);
    r[3] = (int)__builtin_amdgcn_alignbyte(d4, d3, sh);
    return r;
}

template <int MB>
__device__ __forceinline__ v4i read_a(const uint8_t* vb, int t) {
    uint4 x = *reinterpret_cast<const uint4*>(vb + swz<MCfg<MB>::LS>(t));
    v4i r;
    r[0] = (int)x.x; r[1] = (int)x.y; r[2] = (int)x.z; r[3] = (int)x.w;
    return r;
}

template <int MB>
__global__ void __launch_bounds__(256, 2) k_xcorr_mfma(const XItem* items, XItem one) {
    using C = MCfg<MB>;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];

    const XItem& it = items ? items[blockIdx.z] : one;
    const XPair& p = it.p;
    const int64_t T_start = it.T_start;
    const int64_t item_m = it.item_m;
    const int64_t tile = blockIdx.y;
    if (it.engine != TDE_PATH_MFMA || tile >= it.ntiles) return;
    const int64_t T0 = T_start + tile * C::TL;
    const int64_t T1 = T0 + C::TL - 1;
    // m range where some lag of the tile has both u[m] and v[m + tau] in range
    const int64_t m_lo = T1 < 0 ? -T1 : 0;
    const int64_t m_hi = p.nu < p.nv - T0 ? p.nu : p.nv - T0;
    if (m_hi <= m_lo) return;
    const int64_t Q_lo = (m_lo / 32) * 32;
    const int64_t Q_hi = Q_lo + round_up(m_hi + C::S - Q_lo, 32 * MB);
    const int64_t qa = Q_lo + (int64_t)blockIdx.x * item_m;
    if (qa >= Q_hi) return;
    const int64_t qb = qa + item_m < Q_hi ? qa + item_m : Q_hi;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int lc = lane & 31;
    const int g = lane >> 5;

    v16i acc[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[b][e] = 0;

    Stager<MB> st;
    const int nch = (int)((qb - qa + C::CM - 1) / C::CM);
    st.load(p, T0, qa);
    st.store(lds);
    __syncthreads();

    const int a_off = w * C::TLW + C::S * lc + 16 * g;   // A read offset at step 0
    const int b_off = C::UOFF + 16 * g - lc;             // B_0 read offset at step 0

    for (int c = 0; c < nch; ++c) {
        const int64_t qc = qa + (int64_t)c * C::CM;
        if (c + 1 < nch) st.load(p, T0, qc + C::CM);
        const uint8_t* vb = lds + (c & 1) * C::BUF;
        const uint8_t* ub = vb + C::VW;
        const int64_t rem = (qb - qc) / 32;
        const int nsteps = rem < C::CQ ? (int)rem : C::CQ;

        v4i breg[MB];
#pragma unroll
        for (int b = 1; b < MB; ++b) breg[MB - b] = read_b(ub, b_off - 32 * b);

        for (int s0 = 0; s0 < nsteps; s0 += MB) {
#pragma unroll
            for (int t = 0; t < MB; ++t) {
                const int s = s0 + t;
                v4i a = read_a<MB>(vb, a_off + 32 * s);
                breg[t] = read_b(ub, b_off + 32 * s);
#pragma unroll
                for (int b = 0; b < MB; ++b)
                    acc[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, breg[(t - b + MB) % MB], acc[b], 0, 0, 0);
            }
        }
        if (c + 1 < nch) st.store(lds + ((c + 1) & 1) * C::BUF);
        __syncthreads();
    }

    // accumulator layout: lane (j = lc, g), register e -> row i = 8(e/4) + 4g + e%4
    const int64_t Tw = T0 + (int64_t)w * C::TLW;
    const int64_t L = p.lag_hi - p.lag_lo + 1;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int i = 8 * (e >> 2) + 4 * g + (e & 3);
            const int64_t tau = Tw + lc + 32 * b + (int64_t)C::S * i;
            const int64_t idx = tau - p.lag_lo;
            const int val = acc[b][e];
            if (idx >= 0 && idx < L && val != 0) {
                if (p.r_dtype == TDE_I32)
                    atomicAdd(static_cast<int*>(p.r) + idx, val);
                else
                    atomicAdd(static_cast<unsigned long long*>(p.r) + idx, (unsigned long long)(long long)val);
            }
        }
    }
}

// ----------------------------------------------------------------- host --

namespace {
constexpr int kMB = 4;
}

// Sum over the lag tiles of a pair of the m range each tile walks.
int64_t mfma_total_q(const XPair& p) {
    using C = MCfg<kMB>;
    int64_t lo = p.lag_lo > -(p.nu - 1) ? p.lag_lo : -(p.nu - 1);
    int64_t hi = p.lag_hi < p.nv - 1 ? p.lag_hi : p.nv - 1;
    if (lo > hi) return 0;
    int64_t T_start = floor_div(lo, 16) * 16;
    int64_t ntiles = ceil_div(hi - T_start + 1, C::TL);
    int64_t tot = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        int64_t T0 = T_start + t * C::TL, T1 = T0 + C::TL - 1;
        int64_t m_lo = T1 < 0 ? -T1 : 0;
        int64_t m_hi = p.nu < p.nv - T0 ? p.nu : p.nv - T0;
        if (m_hi <= m_lo) continue;
        int64_t Q_lo = (m_lo / 32) * 32;
        tot += round_up(m_hi + C::S - Q_lo, 32 * kMB);
    }
    return tot;
}

// Tiles of the lag range and the split of each tile's m loop. total_q_hint is
// the summed m range of every pair launched together (to size the split).
void mfma_plan(XItem& it, int64_t total_q_hint) {
    using C = MCfg<kMB>;
    const XPair& p = it.p;
    int64_t lo = p.lag_lo > -(p.nu - 1) ? p.lag_lo : -(p.nu - 1);
    int64_t hi = p.lag_hi < p.nv - 1 ? p.lag_hi : p.nv - 1;
    it.ntiles = 0;
    it.nsplit = 0;
    it.item_m = C::CM;
    it.T_start = 0;
    if (lo > hi) return;
    it.T_start = floor_div(lo, 16) * 16;
    it.ntiles = ceil_div(hi - it.T_start + 1, C::TL);
    int64_t maxq = 0;
    for (int64_t t = 0; t < it.ntiles; ++t) {
        int64_t T0 = it.T_start + t * C::TL, T1 = T0 + C::TL - 1;
        int64_t m_lo = T1 < 0 ? -T1 : 0;
        int64_t m_hi = p.nu < p.nv - T0 ? p.nu : p.nv - T0;
        if (m_hi <= m_lo) continue;
        int64_t Q_lo = (m_lo / 32) * 32;
        int64_t len = round_up(m_hi + C::S - Q_lo, 32 * kMB);
        if (len > maxq) maxq = len;
    }
    // int32 partials: item_m * Ku * Kv < 2^31 (kuv <= 127*127 keeps this >= 131072)
    int64_t cap = ((int64_t)0x7fffffff / p.kuv) / C::CM * C::CM;
    if (cap < C::CM) cap = C::CM;
    // aim for ~2048 work items over the whole launch (256 CUs x 2 groups, 4 deep)
    int64_t want = round_up(ceil_div(total_q_hint, 2048), C::CM);
    if (want < C::CM) want = C::CM;
    it.item_m = want < cap ? want : cap;
    it.nsplit = ceil_div(maxq, it.item_m);
}

int launch_xcorr_mfma(const XItem* items_dev, const XItem& one, int nitems, int64_t max_split,
                      int64_t max_tiles, hipStream_t s) {
    using C = MCfg<kMB>;
    if (max_split == 0 || max_tiles == 0) return TDE_OK;
    static bool attr_set = false;
    if (!attr_set) {
        TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_xcorr_mfma<kMB>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_xcorr_mfma<kMB>, dim3((unsigned)max_split, (unsigned)max_tiles, (unsigned)nitems),
                       dim3(256), C::LDS, s, items_dev, one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
