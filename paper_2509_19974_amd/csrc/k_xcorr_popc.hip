// Algorithm 1, correlation step for ternary codes (sign quantization with sign(0) = 0,
// Section 4.2), exact, on bit planes.
//
// Each code c in {-1, 0, +1} is two bits: nz = (c != 0) and sg = (c < 0). A
// product of two codes is 0 unless both are non-zero, and then -1 exactly
// when the signs differ, so over a 32-sample word
//     sum u[m] v[m + tau] = popc(nzu & nzv') - 2 popc(nzu & nzv' & (sgu ^ sgv'))
// where nzv', sgv' are the v planes shifted by tau bits (v_alignbit on two
// neighbouring words). This replaces the paper's "bit operations" view of the
// integer product (Section 3.2) by direct word-parallel sums.
//
// One thread owns one lag; the 32 lanes of a half-wave share the same pair of
// v words, so the loads are broadcasts. The u words are uniform across the
// block. v planes carry zero padding so no shifted read leaves the buffer.
#include "tde_internal.h"

namespace tde {

// blockIdx.z: pair; each thread clears one word of the pair's plane region.
__global__ void __launch_bounds__(256) k_popc_zero(const XItem* items, XItem one) {
    const XItem& it = items ? items[blockIdx.z] : one;
    if (it.engine != TDE_PATH_POPC) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < it.plane_words) it.planes[k] = 0u;
}

__global__ void __launch_bounds__(256) k_popc_pack(const XItem* items, XItem one, int64_t max_words) {
    (void)max_words;                 // sizes the grid; each pair stops at its own words
    const XItem& it = items ? items[blockIdx.z] : one;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it.engine != TDE_PATH_POPC) return;
    const bool is_v = blockIdx.y == 1;
    const int8_t* q = is_v ? it.p.v : it.p.u;
    const int64_t n = is_v ? it.p.nv : it.p.nu;
    const int64_t nw = is_v ? it.nvw : it.nuw;
    if (((int64_t)blockIdx.x * blockDim.x) >= 32 * nw) return;   // whole block past the planes
    uint32_t* sg = const_cast<uint32_t*>(is_v ? it.vsg : it.usg);
    uint32_t* nz = const_cast<uint32_t*>(is_v ? it.vnz : it.unz);
    int c = (m < n) ? (int)q[m] : 0;
    unsigned long long bn = __ballot(c != 0);
    unsigned long long bs = __ballot(c < 0);
    int lane = threadIdx.x & 63;
    int64_t w = m >> 5;   // lanes 0 and 32 of each wave write one word each
    if ((lane & 31) == 0 && w < nw) {
        nz[w] = lane ? (uint32_t)(bn >> 32) : (uint32_t)bn;
        sg[w] = lane ? (uint32_t)(bs >> 32) : (uint32_t)bs;
    }
}

// blockIdx.x: split of the word loop, blockIdx.y: block of 256 lags, z: pair
__global__ void __launch_bounds__(256) k_xcorr_popc(const XItem* items, XItem one) {
    const XItem& it = items ? items[blockIdx.z] : one;
    const XPair& p = it.p;
    if (it.engine != TDE_PATH_POPC || (int64_t)blockIdx.y >= it.ntiles) return;
    const int64_t tb0 = it.T_start + (int64_t)blockIdx.y * 256;        // block's lag range
    const int64_t tb1 = tb0 + 255;
    const int64_t tau = tb0 + threadIdx.x;
    // word range of u where some lag of the block overlaps v
    int64_t m_lo = tb1 < 0 ? -tb1 : 0;
    int64_t m_hi = p.nu < p.nv - tb0 ? p.nu : p.nv - tb0;
    if (m_hi <= m_lo) return;
    int64_t w_lo = m_lo >> 5;
    int64_t w_hi = (m_hi + 31) >> 5;
    int64_t wa = w_lo + (int64_t)blockIdx.x * it.item_m;
    if (wa >= w_hi) return;
    int64_t wb = wa + it.item_m < w_hi ? wa + it.item_m : w_hi;

    const int64_t aw = floor_div(tau, 32);       // v word offset of the lane's lag
    const uint32_t sh = (uint32_t)(tau & 31);
    const uint32_t* __restrict__ usg = it.usg;
    const uint32_t* __restrict__ unz = it.unz;
    const uint32_t* __restrict__ vsg = it.vsg;
    const uint32_t* __restrict__ vnz = it.vnz;
    uint32_t both_cnt = 0, neg_cnt = 0;
    for (int64_t w = wa; w < wb; ++w) {
        const uint32_t su = usg[w];
        const uint32_t nu = unz[w];
        const int64_t vw = w + aw;
        const uint32_t n_lo = vnz[vw], n_hi = vnz[vw + 1];
        const uint32_t s_lo = vsg[vw], s_hi = vsg[vw + 1];
        const uint32_t nv = __builtin_amdgcn_alignbit(n_hi, n_lo, sh);
        const uint32_t sv = __builtin_amdgcn_alignbit(s_hi, s_lo, sh);
        const uint32_t both = nu & nv;
        both_cnt += __builtin_popcount(both);
        neg_cnt += __builtin_popcount(both & (su ^ sv));
    }
    const int val = (int)both_cnt - 2 * (int)neg_cnt;
    const int64_t idx = tau - p.lag_lo;
    const int64_t L = p.lag_hi - p.lag_lo + 1;
    if (idx >= 0 && idx < L && val != 0) {
        if (p.r_dtype == TDE_I32)
            atomicAdd(static_cast<int*>(p.r) + idx, val);
        else
            atomicAdd(static_cast<unsigned long long*>(p.r) + idx, (unsigned long long)(long long)val);
    }
}

// Workspace layout: [usg | unz | vsg (padded) | vnz (padded)], words.
struct PopcLayout {
    int64_t nuw, nvw, pad_lo, vwords;   // v buffer words incl. padding
    int64_t tau0, nblk;
    size_t bytes;
};

static PopcLayout popc_layout(const XPair& p) {
    PopcLayout L{};
    int64_t lo = p.lag_lo > -(p.nu - 1) ? p.lag_lo : -(p.nu - 1);
    int64_t hi = p.lag_hi < p.nv - 1 ? p.lag_hi : p.nv - 1;
    L.nuw = ceil_div(p.nu, 32);
    L.nvw = ceil_div(p.nv, 32);
    if (lo > hi) return L;
    L.tau0 = floor_div(lo, 32) * 32;
    L.nblk = ceil_div(hi - L.tau0 + 1, 256);
    int64_t tau_max = L.tau0 + 256 * L.nblk - 1;
    // v word index = w + floor(tau/32) (+1), w in [0, nuw)
    int64_t a_min = floor_div(L.tau0, 32), a_max = floor_div(tau_max, 32);
    L.pad_lo = a_min < 0 ? -a_min : 0;
    int64_t top = L.nuw + a_max + 2;
    if (top < L.nvw) top = L.nvw;
    L.vwords = L.pad_lo + top;
    L.bytes = align_bytes(2 * L.nuw * 4) + 2 * align_bytes(L.vwords * 4);
    return L;
}

size_t popc_ws_bytes(const XPair& p) { return popc_layout(p).bytes; }

void popc_plan(XItem& it, void* ws) {
    PopcLayout L = popc_layout(it.p);
    it.T_start = L.tau0;
    it.ntiles = L.nblk;
    it.nuw = L.nuw;
    it.nvw = L.nvw;
    uint8_t* base = static_cast<uint8_t*>(ws);
    uint32_t* usg = reinterpret_cast<uint32_t*>(base);
    uint32_t* vsg = reinterpret_cast<uint32_t*>(base + align_bytes(2 * L.nuw * 4));
    uint32_t* vnz = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(vsg) + align_bytes(L.vwords * 4));
    it.planes = usg;
    it.plane_words = (int64_t)(L.bytes / 4);
    it.usg = usg;
    it.unz = usg + L.nuw;
    it.vsg = vsg + L.pad_lo;
    it.vnz = vnz + L.pad_lo;
    // split the word loop so that a launch has enough blocks
    int64_t want_items = L.nblk ? ceil_div(2048, L.nblk) : 1;
    int64_t wpi = ceil_div(L.nuw, want_items);
    if (wpi < 64) wpi = 64;
    it.item_m = wpi;
    it.nsplit = L.nblk ? ceil_div(L.nuw, wpi) : 0;
}

// The padded v planes must be zero outside the packed words: the caller
// zeroes the plane region of the workspace before packing.
int launch_popc_pack(const XItem* items_dev, const XItem& one, int nitems, int64_t max_words, hipStream_t s) {
    if (max_words == 0) return TDE_OK;
    hipLaunchKernelGGL(k_popc_pack, dim3((unsigned)ceil_div(max_words * 32, 256), 2, (unsigned)nitems), dim3(256),
                       0, s, items_dev, one, max_words);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_popc_zero(const XItem* items_dev, const XItem& one, int nitems, int64_t max_words, hipStream_t s) {
    if (max_words == 0 || nitems == 0) return TDE_OK;
    hipLaunchKernelGGL(k_popc_zero, dim3((unsigned)ceil_div(max_words, 256), 1, (unsigned)nitems), dim3(256), 0, s,
                       items_dev, one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_xcorr_popc(const XItem* items_dev, const XItem& one, int nitems, int64_t max_split,
                      int64_t max_tiles, hipStream_t s) {
    if (max_split == 0 || max_tiles == 0) return TDE_OK;
    hipLaunchKernelGGL(k_xcorr_popc, dim3((unsigned)max_split, (unsigned)max_tiles, (unsigned)nitems), dim3(256),
                       0, s, items_dev, one);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
