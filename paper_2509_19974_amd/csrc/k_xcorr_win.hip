// Algorithm 1, correlation step restricted to proposed lag windows: the exact integer
// correlation r[tau] = sum_m u[m] v[m + tau] (Eq. (1)) over one window of 256
// consecutive lags per workgroup, on the int8 matrix cores
// (v_mfma_i32_16x16x64_i8, int32 accumulation), with the window's
// (max, smallest lag, count) triple as the only output.
//
// A window tile holds tau = T0 + j + 16 i (i, j < 16). With steps of 64 in m:
//     A[i][k] = v[q + T0 + 16 i + k]     (rows 16 bytes apart)
//     B[k][j] = u[q + k - j]             (Hankel in (k, j))
//     C[i][j] += sum_k A[i][k] B[k][j]   collects u[m] v[m + tau], m = q + k - j
// For each j the steps q = Qa, Qa + 64, ... cover m in [Qa - j, Qb - j) once,
// so Qa <= first m and Qb >= last m + 16 make every sum complete; samples
// outside the signals are staged as 0 (finite support, Section 2.2).
//
// The 4 waves of a workgroup take a quarter of the steps each, staging their
// own chunk of u and v in LDS; partial tiles meet in LDS in int64. Each
// wave's int32 sum covers at most a quarter of the m range, which the host
// keeps below (2^31 - 1) / (Ku Kv) values.
#include "tde_internal.h"

namespace tde {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWinSteps = 32;                   // steps of 64 m per staged chunk
constexpr int kWinCM = 64 * kWinSteps;          // m per chunk
constexpr int kWinV = kWinCM + 256 + 64;        // v bytes of a chunk (+ one step ahead)
constexpr int kWinU = kWinCM + 64 + 32;         // u bytes: [q0 - 16, q0 + CM + 80)
constexpr int kWinWave = kWinV + kWinU;

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

// grid (npairs * topk): workgroup -> (pair, slot). Pairs whose margin is
// below theta (full-range fallback) are skipped.
__global__ void __launch_bounds__(256) k_xcorr_win(const XItem* items, const int32_t* top, const float* margin,
                                                   float theta, int topk, int nb, ArgPart* parts) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[4 * kWinWave];
    __shared__ unsigned long long red[256];
    __shared__ Tri sh[4];
    const int pair = blockIdx.x / topk, slot = blockIdx.x % topk;
    if (!(margin[pair] >= theta)) return;          // fallback pair (also NaN)
    const XItem& it = items[pair];
    const XPair& p = it.p;
    const int bin = top[(int64_t)pair * topk + slot];
    const int64_t T0 = (int64_t)(bin - nb / 2) * 256;
    // m range of the tile (zero outside the signals)
    const int64_t m_lo = T0 + 255 < 0 ? -(T0 + 255) : 0;
    int64_t m_hi = p.nu < p.nv - T0 ? p.nu : p.nv - T0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v4i acc = {0, 0, 0, 0};
    if (m_hi > m_lo) {
        const int64_t Qa = floor_div(m_lo, 64) * 64;
        const int64_t Qb = ceil_div(m_hi + 15, 64) * 64;
        const int64_t nsteps = (Qb - Qa) / 64;
        const int64_t per = ceil_div(nsteps, 4);
        const int64_t sa = w * per, sb = sa + per < nsteps ? sa + per : nsteps;
        uint8_t* vb = lds + w * kWinWave;
        uint8_t* ub = vb + kWinV;
        const int r = lane & 15, g = lane >> 4;
        const int a_off = 16 * r + 16 * g;                 // A row r, k bytes 16 g .. 16 g + 15
        const int b_off = 16 + 16 * g - r;                 // u[q + 16 g - r ...] relative to q0 - 16
        for (int64_t s0 = sa; s0 < sb; s0 += kWinSteps) {
            const int64_t q0 = Qa + 64 * s0;
            const int ns = (int)(sb - s0 < kWinSteps ? sb - s0 : kWinSteps);
            // stage v[q0 + T0, + kWinV) and u[q0 - 16, + kWinU)
            for (int e = lane; e < kWinV / 16; e += 64)
                *reinterpret_cast<uint4*>(vb + 16 * e) = ld16(p.v, p.nv, q0 + T0 + 16 * e);
            for (int e = lane; e < kWinU / 16; e += 64)
                *reinterpret_cast<uint4*>(ub + 16 * e) = ld16(p.u, p.nu, q0 - 16 + 16 * e);
            for (int s = 0; s < ns; ++s) {
                const uint4 av = *reinterpret_cast<const uint4*>(vb + 64 * s + a_off);
                const int bo = 64 * s + b_off;
                const uint32_t* bw = reinterpret_cast<const uint32_t*>(ub + (bo & ~3));
                uint32_t d[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) d[k] = bw[k];
                const uint32_t sh8 = (uint32_t)(bo & 3);
                v4i a, b;
                a[0] = (int)av.x;
                a[1] = (int)av.y;
                a[2] = (int)av.z;
                a[3] = (int)av.w;
#pragma unroll
                for (int k = 0; k < 4; ++k) b[k] = (int)__builtin_amdgcn_alignbyte(d[k + 1], d[k], sh8);
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc, 0, 0, 0);
            }
        }
    }
    // partial tiles meet in LDS; output layout: lane -> column j = lane % 16,
    // rows 4 (lane / 16) + e
    red[threadIdx.x] = 0ull;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = 4 * (lane >> 4) + e, j = lane & 15;
        if (acc[e]) atomicAdd(&red[16 * i + j], (unsigned long long)(long long)acc[e]);
    }
    __syncthreads();
    // lag index of red[16 i + j] is T0 + j + 16 i - lag_lo
    const int k = threadIdx.x;
    const int64_t idx = T0 + k - p.lag_lo;
    Tri t{INT64_MIN, INT64_MAX, 0};
    if (idx >= 0 && idx <= p.lag_hi - p.lag_lo) t = Tri{(int64_t)red[k], idx, 1};
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Tri u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
        t = tjoin(t, u);
    }
    if (lane == 0) sh[w] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        const Tri a = tjoin(tjoin(sh[0], sh[1]), tjoin(sh[2], sh[3]));
        parts[blockIdx.x] = ArgPart{a.v, a.i, a.c};
    }
}

int launch_xcorr_win(const XItem* items_dev, int npairs, const int32_t* top, const float* margin, float theta,
                     int topk, int nb, ArgPart* parts, hipStream_t s) {
    if (npairs == 0) return TDE_OK;
    hipLaunchKernelGGL(k_xcorr_win, dim3(npairs * topk), dim3(256), 0, s, items_dev, top, margin, theta, topk, nb,
                       parts);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
