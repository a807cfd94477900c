// Internal declarations shared by the HIP kernels and the C-ABI layer of
// libtde.so. Nothing here is part of the public interface (include/tde.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

#include "../../include/tde.h"
#include "exact_sum.h"

namespace tde {

// ------------------------------------------------------------- errors --
int set_error(int status, const char* fmt, ...);
#define TDE_HIP_CHECK(expr)                                                          \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::tde::set_error(TDE_ERR_HIP, "%s failed: %s (%s:%d)", #expr,     \
                                    hipGetErrorString(e_), __FILE__, __LINE__);      \
    } while (0)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
// floor division for possibly negative a (b > 0)
__host__ __device__ inline int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
inline size_t align_bytes(size_t a) { return (a + 255) & ~size_t(255); }

// Loads through the global address space. Pointers fetched from descriptors
// are generic, and generic (flat) loads also count in the LDS wait counter,
// so a prefetch issued that way would stall every later LDS wait until it
// lands; these keep them on the vector-memory counter only.
typedef unsigned int tde_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gload16(const void* p) {
    const tde_u32x4 v = *(const __attribute__((address_space(1))) tde_u32x4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t gload_u8(const int8_t* p) {
    return (uint32_t)(*(const __attribute__((address_space(1))) uint8_t*)p);
}

// A workgroup barrier that orders LDS accesses only: it waits for the wave's
// LDS operations, not for its outstanding global loads and stores, which
// __syncthreads() would also drain.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------ FP4 / FP6 code packing --
// Packed codes for the matrix-core engine's FP4 (E2M1) and FP6 (E2M3)
// operands: W bits per code, code t of a 16-code unit at bits W t of its
// W/2 dwords (the instruction's operand layout). A signal's packed array
// holds ceil(n/16) units, the last one zero-padded.
// Four int8 codes (|q| <= 7, resp. 3) -> four bytes holding W-bit codes:
// sign bit W-1, magnitude code from a byte table (v_perm_b32 as an 8-entry
// lookup), no carries between bytes.
template <int W>
__device__ __forceinline__ uint32_t fp_bytes(uint32_t x) {
    const uint32_t s = (x >> 7) & 0x01010101u;
    const uint32_t a = (x ^ (s * 0xffu)) + s;      // |q| per byte
    // E2M3: 0 1 2 3 4 5 6 7 -> 000000 001000 010000 010100 011000 011010 011100 011110
    // E2M1: 0 1 2 3 (4 . 6 .) -> 0000 0010 0100 0101 (0110 . 0111 .)
    const uint32_t m = W == 6 ? __builtin_amdgcn_perm(0x1e1c1a18u, 0x14100800u, a)
                              : __builtin_amdgcn_perm(0x00070006u, 0x05040200u, a);
    return m | (s << (W - 1));
}

template <int W>
struct Packed16 {
    uint32_t d[W / 2];   // 16 codes
};

// Four bytes of W-bit codes -> their 4W bits, code e at bits W e.
template <int W>
__device__ __forceinline__ uint32_t fp_bits4(uint32_t t) {
    if constexpr (W == 4) {
        t = (t | (t >> 4)) & 0x00ff00ffu;
        return (t | (t >> 8)) & 0x0000ffffu;
    } else {
        t = (t & 0x003f003fu) | ((t >> 2) & 0x0fc00fc0u);
        return (t & 0xfffu) | ((t >> 4) & 0xfff000u);
    }
}

// 16 int8 codes (a uint4, sample order) -> one packed unit.
template <int W>
__device__ __forceinline__ Packed16<W> fp_pack16(uint4 x) {
    const uint32_t z0 = fp_bits4<W>(fp_bytes<W>(x.x)), z1 = fp_bits4<W>(fp_bytes<W>(x.y));
    const uint32_t z2 = fp_bits4<W>(fp_bytes<W>(x.z)), z3 = fp_bits4<W>(fp_bytes<W>(x.w));
    Packed16<W> o;
    if constexpr (W == 4) {
        o.d[0] = z0 | (z1 << 16);
        o.d[1] = z2 | (z3 << 16);
    } else {
        o.d[0] = z0 | (z1 << 24);
        o.d[1] = (z1 >> 8) | (z2 << 16);
        o.d[2] = (z2 >> 16) | (z3 << 8);
    }
    return o;
}

// Fragments of the FP4/FP6 matrix instruction v_mfma_scale_f32_32x32x64_f8f6f4
// (scale 1): a lane holds row (A) or column (B) l mod 32 and k = 32 (l / 32)
// .. + 31, code t at bits W t of its W dwords; the 32 x 32 fp32 result
// has the int8 instruction's layout (lane j + 32 g, register e: row
// 8 (e / 4) + 4 g + (e mod 4), column j).
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Operand format codes of the matrix-core engine (the instruction's own).
constexpr int kFmtI8 = 0;      // (the instruction would read 0 as FP8; int8 items never use it)
constexpr int kFmtF6 = 2;
constexpr int kFmtF4 = 4;

// 16-code unit g of a packed array of n codes (zeros outside the signal).
template <int W>
__device__ __forceinline__ Packed16<W> load_unit(const uint32_t* pk, int64_t n, int64_t g) {
    Packed16<W> o;
    if (g >= 0 && 16 * g < n) {
        const __attribute__((address_space(1))) uint32_t* p =
            (const __attribute__((address_space(1))) uint32_t*)(pk + (W / 2) * g);
#pragma unroll
        for (int k = 0; k < W / 2; ++k) o.d[k] = p[k];
    } else {
#pragma unroll
        for (int k = 0; k < W / 2; ++k) o.d[k] = 0u;
    }
    return o;
}

// A fragment: 32 codes of one row (16 or 24 bytes, 16- resp. 8-byte aligned).
template <int W>
__device__ __forceinline__ v8i read_a_fp(const uint8_t* p) {
    v8i r = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (W == 4) {
        const uint4 x = *reinterpret_cast<const uint4*>(p);
        r[0] = (int)x.x; r[1] = (int)x.y; r[2] = (int)x.z; r[3] = (int)x.w;
    } else {
        const uint2* q = reinterpret_cast<const uint2*>(p);
        const uint2 x = q[0], y = q[1], z = q[2];
        r[0] = (int)x.x; r[1] = (int)x.y; r[2] = (int)y.x; r[3] = (int)y.y; r[4] = (int)z.x; r[5] = (int)z.y;
    }
    return r;
}

template <int W>
struct BWin {
    uint32_t d[2 * W + 1];
};

template <int W>
__device__ __forceinline__ BWin<W> read_bwin(const uint32_t* dw) {
    BWin<W> r;
#pragma unroll
    for (int k = 0; k < 2 * W + 1; ++k) r.d[k] = dw[k];
    return r;
}

// window bits [32 r + sh, ...): B_1 = dwords 0 .. W-1, B_0 = dwords W .. 2W-1
template <int W>
__device__ __forceinline__ void split_bwin(const BWin<W>& r, uint32_t sh, v8i& b1, v8i& b0) {
    b1 = v8i{0, 0, 0, 0, 0, 0, 0, 0};
    b0 = v8i{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < W; ++k) {
        b1[k] = (int)__builtin_amdgcn_alignbit(r.d[k + 1], r.d[k], sh);
        b0[k] = (int)__builtin_amdgcn_alignbit(r.d[W + k + 1], r.d[W + k], sh);
    }
}

// One B fragment (32 codes) per lane: W + 1 dwords from dw, shifted by sh bits.
template <int W>
struct BPiece {
    uint32_t d[W + 1];
};

template <int W>
__device__ __forceinline__ BPiece<W> read_piece(const uint32_t* dw) {
    BPiece<W> r;
#pragma unroll
    for (int k = 0; k < W + 1; ++k) r.d[k] = dw[k];
    return r;
}

template <int W>
__device__ __forceinline__ v8i split_piece(const BPiece<W>& r, uint32_t sh) {
    v8i b = v8i{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < W; ++k) b[k] = (int)__builtin_amdgcn_alignbit(r.d[k + 1], r.d[k], sh);
    return b;
}

template <int W>
__device__ __forceinline__ v16f mfma_fp(const v8i& a, const v8i& b, const v16f& c) {
    constexpr int F = W == 4 ? kFmtF4 : kFmtF6;
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, F, F, 0, 127, 0, 127);
}

// Largest code magnitude of a b-bit quantizer (sign: ternary, K = 1).
inline int kmax_of_bits(int bits) { return bits == 1 ? 1 : (1 << (bits - 1)) - 1; }

// ------------------------------------------------------------ quantize --
// One signal to quantize (Algorithm 1, quantization step).
struct QSig {
    const float* x;
    int64_t n;
    int8_t* q;
    tde_qstat* stat;      // may be null
    double* gsum;         // quantize_gsum_doubles(n) doubles of scratch (auto scale only)
    float* inv_out;       // where the scale in use is written (device)
    int64_t blk_base;     // prefix of ceil(n/kQuantBlock) over the signals before it
    float inv_fixed;      // > 0: caller-supplied scale
    int32_t bits;
    uint16_t* dec;        // optional: n/16 bf16 block means times scale * dec_mul (n a multiple of 16)
    float dec_mul;
    // non-uniform map: code = sign(z) #{k < nthr : |z| > thr[k]}, z = fl32(x inv);
    // nthr = 0 is the uniform map clamp(rint(z), -K, K)
    int32_t nthr;
    float thr[7];
    // optional: the codes packed for the FP4/FP6 matrix-core operands (pk_bits
    // 4 or 6; ceil(n/16) units, the last zero-padded)
    uint32_t* pk;
    int32_t pk_bits;
    // 1: only the packed codes are stored (nothing reads the int8 codes; the
    // statistics still count them)
    int32_t skip_q;
    // 1: the statistics keep only the non-finite and zero counts (sum_q and
    // sum_q2 stay 0), all that the batch call's flags need
    int32_t stat_lite;
};
// z-unit cell boundaries (ascending, K of them) of the non-uniform quantizer
// `kind` (TDE_QUANT_MULAW, TDE_QUANT_GAUSS) for bits 2 or 4; returns K, or 0
// for other arguments
int quant_table(int kind, int bits, float* out);

constexpr int kQuantBlock = 4096;   // samples per quantize workgroup (256 threads x 16)
int64_t quantize_gsum_doubles(int64_t n);
// Queue scale (if needed) + quantization of nsig signals. `sigs_dev` holds the
// descriptors in device memory when nsig > 1; for nsig == 1 `one` is used.
// write_flags: also fill tde_qstat::flags (a separate small launch; the batch
// path derives the flags from the counts where it needs them).
// zero_me (may be null): nzero ints that later kernels of the call expect at 0.
// min_n, max_n: bounds of the signal lengths (0, 0 when unknown); when every
// signal has 1 .. 262144 samples the scale is finished inside the quantize
// kernel instead of a separate launch. When min_n == max_n >= 1 and the
// descriptors are consecutive (blk_base = i ceil(n/kQuantBlock)), a block finds
// its signal by a division instead of a search.
int launch_quantize(const QSig* sigs_dev, const QSig& one, int nsig, int64_t total_blocks, bool need_scale,
                    bool write_flags, int* zero_me, int nzero, hipStream_t s, int64_t min_n = 0, int64_t max_n = 0);

// Result flags of a pair from the statistics of its two signals.
__device__ inline int peak_flags(const tde_qstat* sx, int64_t nx, const tde_qstat* sy, int64_t ny) {
    int f = 0;
    if ((sx && (sx->flags & TDE_FLAG_SCALE_EXACT)) || (sy && (sy->flags & TDE_FLAG_SCALE_EXACT)))
        f |= TDE_FLAG_SCALE_EXACT;
    if (sx) {
        if (sx->n_nonfinite) f |= TDE_FLAG_NONFINITE_X;
        if (sx->n_zero == nx) f |= TDE_FLAG_ZERO_X;
    }
    if (sy) {
        if (sy->n_nonfinite) f |= TDE_FLAG_NONFINITE_Y;
        if (sy->n_zero == ny) f |= TDE_FLAG_ZERO_Y;
    }
    return f;
}

// -------------------------------------------------------------- argmax --
struct ArgPart {          // (max, smallest index, count) of a run of r
    int64_t vmax;
    int64_t idx;
    int64_t cnt;
};

struct ArgSeg {           // one r array to reduce
    const void* r;
    int64_t L;
    int64_t lag_lo;
    int64_t part_base;    // first ArgPart slot of this segment
    int32_t nparts;
    int32_t dtype;
    tde_peak* out;
    const tde_qstat* stat_x;   // flags source (may be null)
    const tde_qstat* stat_y;
    int64_t nx, ny;            // signal lengths (for the all-zero flags)
};

constexpr int kArgChunk = 8192;   // r elements per partial block
int launch_argmax(const ArgSeg* segs_dev, const ArgSeg& one, int nseg, int64_t total_parts,
                  ArgPart* parts, hipStream_t s);

// ---------------------------------------------------------------- xcorr --
// One exact integer correlation r = u * v over [lag_lo, lag_hi].
struct XPair {
    const int8_t* u;
    const int8_t* v;
    int64_t nu, nv;
    int64_t lag_lo, lag_hi;
    void* r;              // lag_hi - lag_lo + 1 elements
    int32_t r_dtype;
    int32_t kuv;          // kmax_u * kmax_v
    int32_t kmax;         // max(kmax_u, kmax_v): selects the operand format of the MFMA engine
    int32_t pad0;
    // FP4/FP6 operands: u and v packed (ceil(n/16) units each), required by
    // items of those formats
    const uint32_t* upk;
    const uint32_t* vpk;
};
// int8 codes -> packed W-bit codes (W = 4 or 6) for the FP operand formats
int launch_pack_fp(const int8_t* q, int64_t n, uint32_t* pk, int W, hipStream_t s);
inline size_t packed_bytes(int64_t n, int W) { return (size_t)((n + 15) / 16) * 2 * W; }

// fill r with zeros (a kernel, never a memset node)
int launch_zero(void* p, size_t bytes, hipStream_t s);

// One correlation job for a batched engine launch: the pair plus its plan.
struct XItem {
    XPair p;
    int32_t engine;       // TDE_PATH_MFMA or TDE_PATH_POPC: kernels skip other items
    int32_t mb;           // MFMA engine: accumulator tiles per wave
    int64_t T_start;      // first lag of tile 0
    int64_t item_m;       // bit-plane engine: u words per split item
    int64_t ntiles;       // lag tiles of this pair
    int64_t nsplit;       // bit-plane engine: split items per tile
    // MFMA engine
    int32_t wide;         // tile sums may exceed int32: reduce in int64
    int32_t segmented;    // tiles cut into several items: r by atomics, no triples
    int32_t fused;        // argmax from tile triples (no r array needed)
    int32_t fmt;          // MFMA operand format (kFmtI8, kFmtF6, kFmtF4)
    int64_t part_base;    // first tile-triple slot of this pair
    int64_t out_v, out_i, out_c;   // triple of the lags no tile covers (r = 0)
    const tde_qstat* stat_x;
    const tde_qstat* stat_y;
    tde_peak* peak;
    // bit-plane engine only
    const uint32_t* usg;
    const uint32_t* unz;
    const uint32_t* vsg;  // word of sample 0 (zero padding before and after)
    const uint32_t* vnz;
    int64_t nuw;          // u words
    int64_t nvw;          // v words
    uint32_t* planes;     // the pair's whole plane region (zeroed before packing)
    int64_t plane_words;  // its size in 32-bit words
    // learned mode: the pair's proposal margin; at or above theta the result
    // comes from the nwin window triples, below it from the full range
    const float* margin;  // null outside learned mode
    float theta;
    int32_t nwin;
    const ArgPart* win_parts;
    int32_t win_w;        // learned mode: 4 or 6, windows on FP operands of that width; 0, on int8
    // learned mode with the fallback planned on the device: the pair's
    // unsegmented matrix-core items in the static list
    int32_t work_first, work_count;
};

// zero the bit-plane regions of a batch (one launch for every pair)
int launch_popc_zero(const XItem* items_dev, const XItem& one, int nitems, int64_t max_words, hipStream_t s);

// zero the r arrays of a batch
int launch_zero_r(const XItem* items_dev, const XItem& one, int nitems, int64_t max_rbytes, hipStream_t s);

// direct int8-MFMA engine: pairs are cut into lag tiles, each one work item
// (or several segments for very long signals) that a persistent kernel takes
// longest-first.
struct MWork {
    int32_t pair;         // index into the XItem array
    int32_t tile;         // lag tile of the pair
    int64_t qa, qb;       // m range [qa, qb), multiples of 32
    int32_t segmented;
    int32_t mb;           // accumulator tiles per wave of the pair's plan
    int32_t fmt;          // operand format of the pair's plan
    int32_t rslot;        // 0, or k + 1: r is slot k of the learned fallback's pool (not the pair's r)
};
// Operand formats of the matrix-core engine (kFmtI8, kFmtF6, kFmtF4 above).
// Codes with |q| <= 3 are exact in FP4 (E2M1), |q| <= 7 in FP6 (E2M3); both
// run the f8f6f4 matrix instruction at twice the int8 rate.
// sets fmt, mb, T_start, ntiles, wide, segmented, outside triple; allow_fp =
// false keeps int8 operands whatever the code range
void mfma_plan_pair(XItem& it, bool allow_fp = true);
int mfma_choose_fmt(int kmax, bool allow_fp);   // kFmt* for codes up to kmax
int64_t mfma_total_q(const XItem& it);          // summed m range of its tiles
int64_t mfma_count_items(const XItem& it);
void mfma_items(const XItem& it, int pair, std::vector<MWork>& out);
// Launch that runs an item: the 4-block one for int8 4-block items and every
// FP item, the 8-block one for int8 8-block items.
inline int mfma_launch_of(int fmt, int mb) { return fmt == kFmtI8 && mb == 8 ? 8 : 4; }
void mfma_sort_items(std::vector<MWork>& w);
// work_dev: nwork items sorted by mfma_sort_items, the first n4 of them with
// mb = 4. tile_parts may be null (no triples written); counters_dev: 2 ints
// of scratch, reset here unless an earlier kernel of the call already did.
int choose_mb(const XPair& p);
int launch_xcorr_mfma(const XItem* items_dev, const MWork* work_dev, int nwork, int* counters_dev,
                      bool counters_zeroed, ArgPart* tile_parts, int num_cu, hipStream_t s, int n4,
                      const int* nwork_dev = nullptr, uint8_t* rpool = nullptr, int64_t slot_bytes = 0);
// peaks of the fused pairs from their tile triples
int launch_tiles_final(const XItem* items_dev, const XItem& one, int npairs, const ArgPart* tile_parts,
                       hipStream_t s);
// Learned mode, fallback planned on the device (graph-safe, no host
// decision): the pairs whose margin is below the threshold get their
// matrix-core items in a work list whose length the engine reads from
// ctl[1]. When few pairs fall back (at most kFbSlots, fewer items than
// `target`), each item is cut into up to kFbMaxSplit segments along m that
// add into slot k of rpool (ctl[0] pairs, slots[k] = pair, the item's
// rslot = k + 1), so that the segments fill the device; launch_fb_zero
// clears those slots first and launch_fb_argmax writes their peaks after
// the engine (over the peaks launch_tiles_final wrote from unused tile
// triples). The descriptors are never written during a call: what the
// planner writes is read back with device-scope loads, never through the
// scalar cache that earlier kernels of the call may have filled.
constexpr int kFbSlots = 64, kFbMaxSplit = 16;
int launch_fb_plan(const XItem* items_dev, int npairs, const MWork* swork, MWork* dwork, int* ctl, int* slots,
                   int target, hipStream_t s);
int launch_fb_zero(const XItem* items_dev, const int* ctl, const int* slots, uint8_t* rpool, int64_t slot_bytes,
                   hipStream_t s);
// parts: kFbSlots * 64 ArgPart of scratch
int launch_fb_argmax(const XItem* items_dev, const int* ctl, const int* slots, const uint8_t* rpool,
                     int64_t slot_bytes, ArgPart* parts, hipStream_t s);

// bit-plane engine for ternary codes
size_t popc_ws_bytes(const XPair& p);
// fills the plane pointers of `it` (inside ws) and its plan
void popc_plan(XItem& it, void* ws);
int launch_popc_pack(const XItem* items_dev, const XItem& one, int nitems, int64_t max_words, hipStream_t s);
int launch_xcorr_popc(const XItem* items_dev, const XItem& one, int nitems, int64_t max_split,
                      int64_t max_tiles, hipStream_t s);

// int8 copy helper
int launch_copy_bytes(void* dst, const void* src, size_t n, hipStream_t s);

// windowed exact engine (learned mode), windows of 256 lags: formats bit 0
// launches the int8 kernel (a workgroup per window) for pairs with win_w = 0,
// bits 1 and 2 the FP6 and FP4 kernels (a workgroup per pair, topk <= 8)
// for pairs with win_w = 6 and 4
int launch_xcorr_win(const XItem* items_dev, int npairs, const int32_t* top, const float* margin, float theta,
                     int topk, int nb, ArgPart* parts, hipStream_t s, int formats);

// tie refinement (Algorithm 1, tie-refinement step): scratch of one call,
// every array sized for max_ties lags except hits (kRefineMaxChunks per-chunk
// counts of the collect) and limbs (kExactLimbs int64 per lag)
constexpr int kRefineMaxChunks = 4096;
struct RefineWs {
    int64_t* lags;        // collected tied lags
    double* vals;         // float64 tree sums of the real correlation
    double* errs;         // their error bounds
    int* cand;            // lags (indices into lags) that still need exact sums
    int* ncand;
    int* count;           // tied lags in r
    int* hits;
    int64_t* limbs;       // exact sums of the candidates
};
RefineWs refine_ws_carve(void* ws, int max_ties, size_t* bytes);
int launch_refine(const float* x, int64_t nx, const float* y, int64_t ny, const void* r, int dtype, int64_t lag_lo,
                  int64_t L, tde_peak* peak, int max_ties, const RefineWs& w, hipStream_t s);

// ---------------------------------------------------------- auto engine --
// HIP device of a context.
int ctx_device(const tde_ctx* ctx);
int ctx_num_cu(const tde_ctx* ctx);
// Engine for TDE_PATH_AUTO (tuning table, else the built-in cost model).
int auto_engine(int64_t nu, int64_t nv, int kuv, int kmax, int64_t lag_lo, int64_t lag_hi);
// Accumulator blocks per matrix-core tile (4 or 8) for a correlation's
// bucket: the tuner's forced value while it measures, else the tuning
// table's entry, else 0 (the built-in rule decides).
int tuned_tile_blocks(int64_t nu, int64_t nv, int kuv, int64_t lag_lo, int64_t lag_hi);

// ----------------------------------------------------------------- NTT --
// Number-theoretic-transform engine (two primes + CRT), for long signals.
constexpr int kNttRow = 4096;      // row length of the four-step split
constexpr int kNttC1 = 16;         // columns per forward-column workgroup
constexpr int kNttMinLog = 13, kNttMaxLog = 23;
constexpr int kNttK1Per = 16 * 2048 / 1024;  // forward-column codes per thread, at most
constexpr int kNttK3Per = 32768 / 1024;   // inverse-column residues per thread, at most

struct NttPlan {
    int log_n;            // transform length n = 2^log_n
    int nprimes;          // 1 or 2
    int64_t jlo, jhi;     // positions j = tau + nu - 1 computed (empty if jlo > jhi)
    int wc3;              // columns per inverse-column workgroup
    int ntiles;           // inverse-column workgroups = argmax triples
};

struct NttGroup {         // passed by value: everything shared by a launch
    uint32_t* tab;        // twiddle tables (device), nprimes x (n1 + 8192) (w, Shoup quotient) word pairs
    int log_n, log_n1, n1, nprimes, wc3;
    uint32_t p[2], pinv[2], one_m[2], root_m[2], scale_m[2], crt_m;
};

struct NttJob {           // one pair (device descriptor)
    const int8_t* u;
    const int8_t* v;
    int64_t nu, nv, lag_lo;
    int64_t jlo, jhi;
    void* r;              // may be null
    int32_t r_dtype;
    int32_t pad;
    uint32_t* res;        // 2 x nprimes x n residues
    ArgPart* parts;       // ntiles triples, or null
};

// false when the transform would exceed 2^kNttMaxLog
bool ntt_plan(int64_t nu, int64_t nv, int kuv, int64_t lag_lo, int64_t lag_hi, NttPlan& P);
size_t ntt_tab_words(const NttPlan& P);
size_t ntt_res_bytes(const NttPlan& P);
NttGroup ntt_group(const NttPlan& P, uint32_t* tab);
// All jobs share the group's n and prime count.
int launch_ntt(const NttGroup& g, const NttJob* jobs_dev, int njobs, hipStream_t s);

// ----------------------------------------------------------------- CNN --
// Learned lag-window proposer (fixed architecture: 4 conv layers of 32
// channels, kernel 9, average pooling 2, correlation head).
constexpr int kCnnC = 32, kCnnK = 9, kCnnLayers = 4, kCnnMaxTop = 16;

struct CnnSig {           // one signal to decimate
    const float* x;       // 16 ld samples
    const float* inv;     // quantizer scale (device) or null
    float scale_mul;      // scale = *inv * scale_mul (or scale_mul alone)
};

struct CnnNet {
    int ld;               // decimated input length (multiple of 256)
    int nb;               // bins (multiple of 64, at most 2 ld / 16)
    int nparams;
    const void* frag;     // packed matrix-core weight fragments (device), 3 x 18 x 64 x 16 bytes
};
constexpr size_t kCnnFragBytes = 2 * 3 * 18 * 64 * 16;   // fragments of W, then of W / 2

struct CnnActs {          // per layer l: input X_l (x[0] = decimated input), pre-activation Z_l
    uint16_t* x[kCnnLayers + 1];
    uint16_t* z[kCnnLayers];   // null for inference
};

struct CnnGrad {
    float* dx[kCnnLayers + 1];   // gradient of each layer's output (dx[4] = features)
    float* part;                 // per-workgroup weight-gradient partials
    float* grad;                 // flat, parameter layout
    float* dlog;                 // [B][nb]
    float* dalpha;               // [B]
    float* loss;                 // [B]
};

int cnn_param_count(int layers);
size_t cnn_param_offset(int layer);
int launch_cnn_decimate(const CnnSig* sigs, int nsig, int ld, uint16_t* out, hipStream_t s);
int launch_cnn_forward(const CnnNet& net, const float* wc, const uint16_t* xdec, int B, CnnActs& A, float* raw,
                       float* logits, hipStream_t s);
int launch_cnn_topk(const float* logits, int B, int nb, int topk, int32_t* top, float* margin, hipStream_t s);
int launch_cnn_backward(const CnnNet& net, const float* wc, int B, const int32_t* labels, CnnActs& A,
                        const float* raw, const float* logits, CnnGrad& G, hipStream_t s);
int launch_adam(float* p, const float* g, float* m, float* v, float* wc, int n, float lr, int step, hipStream_t s);
int launch_round_copy(const float* p, float* wc, int n, hipStream_t s);
int launch_pack_frags(const float* wc, void* frag, hipStream_t s);
// model accessors and the allocation-free inference used by the batch call
const CnnNet& model_net(const tde_model* M);
int model_device(const tde_model* M);
size_t cnn_infer_bytes(const CnnNet& net, int B);
// Decimates (sigs_dev: 2 B descriptors) or takes xdec, runs the encoder and
// head with activations carved from ws (cnn_infer_bytes), then top-k.
int cnn_infer(const tde_model* M, const uint16_t* xdec_or_null, int B, uint8_t* ws, int topk, int32_t* top,
              float* margin, float* logits_out, hipStream_t s, const CnnSig* sigs_dev);

}  // namespace tde
