// Algorithm 1, argmax step: the argmax of the integer correlation, reported as the
// smallest maximising lag, the maximum and the number of maximisers (Remark 1:
// the quantized correlation may have several peaks).
//
// (max, smallest index, count) triples combine associatively and
// commutatively: the larger max wins; equal maxima keep the smaller index and
// add the counts. Each block reduces a run of r (wave shuffles, then LDS) to a
// partial; one block per segment combines its partials in a fixed order, so
// the result never depends on scheduling.
#include "tde_internal.h"

namespace tde {

struct Tri {
    int64_t v, i, c;
};

__device__ __forceinline__ Tri tri_combine(Tri a, Tri b) {
    if (b.v > a.v) return b;
    if (a.v > b.v) return a;
    Tri r;
    r.v = a.v;
    r.i = a.i < b.i ? a.i : b.i;
    r.c = a.c + b.c;
    return r;
}

__device__ __forceinline__ Tri wave_tri(Tri t) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Tri u;
        u.v = __shfl_xor(t.v, o, 64);
        u.i = __shfl_xor(t.i, o, 64);
        u.c = __shfl_xor(t.c, o, 64);
        t = tri_combine(t, u);
    }
    return t;
}

__device__ __forceinline__ Tri block_tri(Tri t) {
    __shared__ Tri sh[4];
    t = wave_tri(t);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        Tri a = sh[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) a = tri_combine(a, sh[k]);
        sh[0] = a;
    }
    __syncthreads();
    Tri r = sh[0];
    __syncthreads();
    return r;
}

constexpr int64_t kNone = INT64_MIN;

__device__ __forceinline__ const ArgSeg& seg_of(const ArgSeg* segs, int nseg, const ArgSeg& one,
                                                int64_t part, int64_t& local) {
    if (!segs) {
        local = part;
        return one;
    }
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].part_base <= part) lo = mid; else hi = mid - 1;
    }
    local = part - segs[lo].part_base;
    return segs[lo];
}

__global__ void __launch_bounds__(256) k_argmax_partial(const ArgSeg* segs, int nseg, ArgSeg one,
                                                        ArgPart* parts) {
    const int64_t part = blockIdx.x;
    int64_t lp;
    const ArgSeg& s = seg_of(segs, nseg, one, part, lp);
    const int64_t lo = lp * kArgChunk;
    const int64_t hi = lo + kArgChunk < s.L ? lo + kArgChunk : s.L;
    Tri t{kNone, INT64_MAX, 0};
    if (s.dtype == TDE_I32) {
        const int32_t* r = static_cast<const int32_t*>(s.r);
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            Tri u{(int64_t)r[i], i, 1};
            t = tri_combine(t, u);
        }
    } else {
        const int64_t* r = static_cast<const int64_t*>(s.r);
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            Tri u{r[i], i, 1};
            t = tri_combine(t, u);
        }
    }
    t = block_tri(t);
    if (threadIdx.x == 0) parts[part] = ArgPart{t.v, t.i, t.c};
}

__global__ void __launch_bounds__(256) k_argmax_final(const ArgSeg* segs, int nseg, ArgSeg one,
                                                      const ArgPart* parts) {
    (void)nseg;                      // the grid has one workgroup per segment
    const ArgSeg& s = segs ? segs[blockIdx.x] : one;
    Tri t{kNone, INT64_MAX, 0};
    for (int k = threadIdx.x; k < s.nparts; k += blockDim.x) {
        ArgPart p = parts[s.part_base + k];
        t = tri_combine(t, Tri{p.vmax, p.idx, p.cnt});
    }
    t = block_tri(t);
    if (threadIdx.x == 0) {
        const int flags = peak_flags(s.stat_x, s.nx, s.stat_y, s.ny);
        tde_peak pk;
        pk.lag = s.lag_lo + t.i;
        pk.rmax = t.v;
        pk.n_ties = (int32_t)t.c;
        pk.flags = flags;
        *s.out = pk;
    }
}

int launch_argmax(const ArgSeg* segs_dev, const ArgSeg& one, int nseg, int64_t total_parts,
                  ArgPart* parts, hipStream_t s) {
    hipLaunchKernelGGL(k_argmax_partial, dim3((unsigned)total_parts), dim3(256), 0, s, segs_dev, nseg, one,
                       parts);
    hipLaunchKernelGGL(k_argmax_final, dim3(nseg), dim3(256), 0, s, segs_dev, nseg, one, parts);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

// ------------------------------------------------------------ helpers --

__global__ void k_zero(uint32_t* p, size_t nwords) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < nwords; i += stride) p[i] = 0u;
}

__global__ void k_zero_bytes(uint8_t* p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

int launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return TDE_OK;
    uintptr_t a = (uintptr_t)p;
    size_t head = (4 - (a & 3)) & 3;
    if (head > bytes) head = bytes;
    if (head) hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, s, (uint8_t*)p, head);
    size_t words = (bytes - head) / 4;
    if (words) {
        size_t blocks = (words + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)((uint8_t*)p + head), words);
    }
    size_t tail = bytes - head - 4 * words;
    if (tail) hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, s, (uint8_t*)p + head + 4 * words, tail);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

__global__ void k_copy_bytes(uint8_t* d, const uint8_t* src, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = src[i];
}

int launch_copy_bytes(void* dst, const void* src, size_t n, hipStream_t s) {
    if (!n) return TDE_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy_bytes, dim3((unsigned)blocks), dim3(256), 0, s, (uint8_t*)dst,
                       (const uint8_t*)src, n);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde

namespace tde {

// Zero the r arrays of a batch: blockIdx.y selects the item.
__global__ void k_zero_r(const XItem* items, XItem one) {
    const XItem& it = items ? items[blockIdx.y] : one;
    if (!it.p.r) return;
    const int64_t words = (it.p.lag_hi - it.p.lag_lo + 1) * (it.p.r_dtype == TDE_I32 ? 1 : 2);
    uint32_t* r = static_cast<uint32_t*>(it.p.r);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        r[i] = 0u;
}

int launch_zero_r(const XItem* items_dev, const XItem& one, int nitems, int64_t max_rbytes, hipStream_t s) {
    int64_t blocks = ceil_div(max_rbytes / 4, 256 * 4);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_r, dim3((unsigned)blocks, (unsigned)nitems), dim3(256), 0, s, items_dev, one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
