// Algorithm 1, correlation step (Eq. (1) on integer codes), exact, on the int8 matrix
// cores of gfx950 (v_mfma_i32_32x32x32_i8, int32 accumulation), with the
// argmax step taken on chip.
//
// The correlation r[tau] = sum_m u[m] v[m + tau] is a product of a Hankel
// and a Toeplitz matrix. A lag tile is 1024*MB consecutive lags
//     tau = T0 + c + S*i,   c = j + 32 b in [0, S),  S = 32 MB,  i, j in [0, 32)
// held in MB accumulator tiles C_b[i][j] per wave (rows i: coarse lag,
// columns j: fine lag, so the 32 lanes of a tile row hold 32 consecutive
// lags). The k loop walks m in steps of 32:
//     A[i][k]   = v[q + T0 + S i + k]        (rows S bytes apart, 16-byte aligned)
//     B_b[k][j] = u[q + k - j - 32 b]        (Hankel in (k, j))
//     C_b      += A x B_b
// so C_b[i][j] collects u[m] v[m + tau] for m = q + k - j - 32 b. The Hankel
// structure gives B_b(q) = B_0(q - 32 b): each step reads one A and one new B
// fragment for MB matrix instructions; the other MB-1 B fragments are the
// previous steps' B_0, kept in registers.
//
// Work decomposition: a work item is one lag tile of one pair and the whole
// m range that tile needs (or, for very long signals, one segment of it).
// The 4 waves of a workgroup take one quarter of the m range each and run
// independently: each wave stages its own v and u windows in a private LDS
// region, so the main loop has no workgroup barrier. The v window of a
// 128-step chunk (TLW + 4096 bytes) moves by 4096 bytes per chunk and lives in
// a power-of-two ring; every S bytes carry 16 bytes of padding so the 32 rows
// of an A fragment fall into distinct banks. B rows start at arbitrary byte
// offsets and are assembled from 5 dwords with v_alignbyte. Out-of-range
// samples are staged as 0: the finite-length convention of Section 2.2.
//
// At the end of an item the four partial sums meet in LDS (ds_add, 32- or
// 64-bit). The tile then writes r with plain coalesced stores when r is
// requested, and its (max, smallest lag, count) triple (kept in 32-bit for
// int32 tiles), so no r array is needed for the argmax.
// Each wave's partial covers at most floor((2^31-1)/(Ku Kv)) values of m, so
// no int32 accumulator overflows (coefficient bound of Section 3.2); tiles
// whose total may exceed int32 are summed in int64. Segmented tiles add into
// r with integer atomics (exact, order-independent).
//
// The kernel is persistent: workgroups take items from an atomic counter over
// a list sorted longest-first.
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "tde_internal.h"

namespace tde {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

template <int MB>
struct MCfg {
    static constexpr int S = 32 * MB;          // coarse lag stride, A row stride
    static constexpr int LS = MB == 4 ? 7 : 8; // log2(S)
    static constexpr int TLW = 32 * S;         // lags per tile
    static constexpr int CQ = 128;             // k steps per staged chunk
    static constexpr int CM = 32 * CQ;         // m per chunk
    // per-wave v window of a chunk: [0, VW); the last A read (one step ahead)
    // ends at TLW + CM - S + 32 <= VW
    static constexpr int VW = TLW + CM;
    // ring (power of two) >= VW: the new bytes of chunk c+1 are stored only
    // after every read of chunk c (a wave's LDS operations complete in order),
    // and they land on the bytes chunk c + 1 no longer needs
    static constexpr int R = MB == 4 ? 8192 : 16384;
    static_assert(R >= VW, "ring too small");
    static constexpr int VPH = R + 16 * (R / S);       // padded ring bytes
    static constexpr int UOFF = 32 * MB;               // u window starts UOFF before the chunk
    // u window; the last B read (one step ahead) ends at UOFF + CM + 36 <= UW.
    // One buffer: a wave's LDS operations complete in order, so its reads of
    // chunk c are done before its writes for chunk c+1.
    static constexpr int UW = CM + UOFF + 64;
    static constexpr int WAVE_LDS = VPH + UW;
    static constexpr int LDS = 4 * WAVE_LDS;
    static_assert(LDS >= TLW * 8, "reduction area must fit");
    static constexpr int FILL_V = VW / 16;             // 16-byte units
    static constexpr int NEW_V = CM / 16;
    static constexpr int U_UNITS = UW / 16;
    static constexpr int FILL_PER_LANE = (FILL_V + U_UNITS + 63) / 64;
    static constexpr int NEXT_PER_LANE = (NEW_V + U_UNITS + 63) / 64;
};

// ring position -> LDS byte (16 bytes of padding after every S bytes)
template <int MB>
__device__ __forceinline__ int vphys(int p) {
    return p + 16 * (p >> MCfg<MB>::LS);
}

__device__ __forceinline__ uint4 load16_guarded(const int8_t* base, int64_t n, int64_t gi) {
    const int8_t* p = base + gi;
    if (gi >= 0 && gi + 16 <= n && ((((uintptr_t)p) & 15) == 0)) return gload16(p);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (gi + 16 > 0 && gi < n) {
        for (int e = 0; e < 16; ++e) {
            int64_t idx = gi + e;
            uint32_t byte = (idx >= 0 && idx < n) ? gload_u8(base + idx) : 0u;
            w[e >> 2] |= byte << (8 * (e & 3));
        }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// The value itself, hidden from the optimiser: per-lane constants derived
// from it are recomputed where they are used instead of being hoisted out of
// the persistent loop, where they would hold registers for the whole kernel.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// The next work item of the persistent loop, taken from the counter while the
// last chunk of the current item runs (one lane of the workgroup asks), so
// the atomic's round trip overlaps the matrix work. Taking it this late keeps
// the longest-first order of the dynamic schedule.
struct NextItem {
    int* counter;
    bool ask;       // the asking lane, until it has asked
    int v;
    __device__ __forceinline__ void fetch() {
        if (ask) {
            // a lane-varying address as far as the compiler knows: an atomic
            // on a uniform address is rewritten into a form that waits for
            // its result right away
            v = atomicAdd(counter + opaque(0), 1);
            ask = false;
        }
    }
};

// Per-wave staging. Chunk c of a wave covers m steps [qw + c CM, qw + (c+1) CM);
// its v window starts at global v index qw + c CM + T0, at ring byte
// (c CM) mod R. Only the wave itself touches its region.
template <int MB>
struct WaveStager {
    using C = MCfg<MB>;
    uint4 reg[C::NEXT_PER_LANE];
    // the descriptor fields, read once: LDS stores go through generic
    // pointers, after which fields read through the descriptor would be
    // reloaded from memory
    const int8_t* u;
    const int8_t* v;
    int64_t nu, nv;
    __device__ __forceinline__ explicit WaveStager(const XPair& p) : u(p.u), v(p.v), nu(p.nu), nv(p.nv) {}

    __device__ __forceinline__ void fill(int64_t T0, int64_t qw, uint8_t* vb, uint8_t* ub, int lane) {
        lane = opaque(lane);
        const int64_t gv0 = qw + T0;
        const int64_t gu0 = qw - C::UOFF;
        uint4 x[C::FILL_PER_LANE];
#pragma unroll
        for (int k = 0; k < C::FILL_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::FILL_V)
                x[k] = load16_guarded(v, nv, gv0 + 16 * (int64_t)unit);
            else if (unit < C::FILL_V + C::U_UNITS)
                x[k] = load16_guarded(u, nu, gu0 + 16 * (int64_t)(unit - C::FILL_V));
        }
#pragma unroll
        for (int k = 0; k < C::FILL_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::FILL_V)
                *reinterpret_cast<uint4*>(vb + vphys<MB>(16 * unit)) = x[k];
            else if (unit < C::FILL_V + C::U_UNITS)
                *reinterpret_cast<uint4*>(ub + 16 * (unit - C::FILL_V)) = x[k];
        }
    }
    __device__ __forceinline__ void load_next(int64_t T0, int64_t qw, int c, int lane) {
        lane = opaque(lane);
        const int64_t rel0 = (int64_t)(c - 1) * C::CM + C::VW;    // first new window byte
        const int64_t gv0 = qw + T0 + rel0;
        const int64_t gu0 = qw + (int64_t)c * C::CM - C::UOFF;
#pragma unroll
        for (int k = 0; k < C::NEXT_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::NEW_V)
                reg[k] = load16_guarded(v, nv, gv0 + 16 * (int64_t)unit);
            else if (unit < C::NEW_V + C::U_UNITS)
                reg[k] = load16_guarded(u, nu, gu0 + 16 * (int64_t)(unit - C::NEW_V));
        }
    }
    __device__ __forceinline__ void store_next(int c, uint8_t* vb, uint8_t* ub, int lane) {
        lane = opaque(lane);
        const int rel0 = (int)(((int64_t)(c - 1) * C::CM + C::VW) & (C::R - 1));
#pragma unroll
        for (int k = 0; k < C::NEXT_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::NEW_V)
                *reinterpret_cast<uint4*>(vb + vphys<MB>((rel0 + 16 * unit) & (C::R - 1))) = reg[k];
            else if (unit < C::NEW_V + C::U_UNITS)
                *reinterpret_cast<uint4*>(ub + 16 * (unit - C::NEW_V)) = reg[k];
        }
    }
};

// 16 bytes of the u window at a byte offset, read as 5 dwords (issued early)
// and assembled with v_alignbyte (later).
struct BRaw {
    uint32_t d[5];
};

__device__ __forceinline__ BRaw read_b_raw(const uint32_t* dw) {
    BRaw r;
#pragma unroll
    for (int k = 0; k < 5; ++k) r.d[k] = dw[k];
    return r;
}

__device__ __forceinline__ v4i assemble_b(const BRaw& r, uint32_t sh) {
    v4i o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = (int)__builtin_amdgcn_alignbyte(r.d[k + 1], r.d[k], sh);
    return o;
}

__device__ __forceinline__ v4i read_a(const uint8_t* p) {
    uint4 x = *reinterpret_cast<const uint4*>(p);
    v4i r;
    r[0] = (int)x.x; r[1] = (int)x.y; r[2] = (int)x.z; r[3] = (int)x.w;
    return r;
}

// (max, smallest index, count) over a run of lags.
struct Tri64 {
    int64_t v, i, c;
};

__device__ __forceinline__ Tri64 tri_join(Tri64 a, Tri64 b) {
    if (b.v > a.v) return b;
    if (a.v > b.v) return a;
    return Tri64{a.v, a.i < b.i ? a.i : b.i, a.c + b.c};
}

// The m loop of one wave over [qw_a, qw_b) for the tile at T0.
template <int MB>
__device__ __forceinline__ void wave_loop(const XPair& p, int64_t T0, int64_t qw_a, int64_t qw_b, uint8_t* wl,
                                          int lane, v16i* acc, NextItem& nx) {
    using C = MCfg<MB>;
    lane = opaque(lane);
    const int lc = lane & 31;
    const int g = lane >> 5;
    uint8_t* vb = wl;
    uint8_t* ubufs = wl + C::VPH;
    WaveStager<MB> st(p);
    const int nch = (int)((qw_b - qw_a + C::CM - 1) / C::CM);
    st.fill(T0, qw_a, vb, ubufs, lane);

    const int a_off = C::S * lc + 16 * g;             // A read offset at step 0
    const int b_off = C::UOFF + 16 * g - lc;          // B_0 read offset at step 0 (> 0)
    const uint32_t bsh = (uint32_t)(b_off & 3);

    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) st.load_next(T0, qw_a, c + 1, lane);
        else nx.fetch();
        const int base = (int)(((int64_t)c * C::CM) & (C::R - 1));
        const uint32_t* ubw = reinterpret_cast<const uint32_t*>(ubufs) + (b_off >> 2);
        const int64_t rem = (qw_b - qw_a - (int64_t)c * C::CM) / 32;
        const int nsteps = rem < C::CQ ? (int)rem : C::CQ;

        v4i breg[MB];
#pragma unroll
        for (int b = 1; b < MB; ++b) breg[MB - b] = assemble_b(read_b_raw(ubw - 8 * b), bsh);
        // Software pipeline: fragments of step s+1 are read while the matrix
        // instructions of step s run; reading one step past the chunk stays
        // inside the staged windows. Inside a group of MB steps the A rows
        // stay in one padded S-byte block (the ring end is S-aligned), so
        // their LDS offsets are constants. (Unlike the FP loop, each chunk
        // re-reads its history and step 0: carrying them over measured 3%
        // slower here.)
        int p0 = (base + a_off) & (C::R - 1);
        const uint8_t* arow = vb + vphys<MB>(p0);
        v4i a_cur = read_a(arow);
        v4i b_cur = assemble_b(read_b_raw(ubw), bsh);
        for (int s0 = 0; s0 < nsteps; s0 += MB) {
            const int pn = (p0 + C::S) & (C::R - 1);
            const uint8_t* arow_next = vb + vphys<MB>(pn);
#pragma unroll
            for (int t = 0; t < MB; ++t) {
                const int s = s0 + t;
                const v4i a_nxt = read_a(t + 1 < MB ? arow + 32 * (t + 1) : arow_next);
                const BRaw b_raw = read_b_raw(ubw + 8 * (s + 1));
                __builtin_amdgcn_sched_barrier(0);
                breg[t] = b_cur;
#pragma unroll
                for (int b = 0; b < MB; ++b)
                    acc[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_cur, breg[(t - b + MB) % MB], acc[b], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                a_cur = a_nxt;
                b_cur = assemble_b(b_raw, bsh);
                __builtin_amdgcn_sched_barrier(0);
            }
            p0 = pn;
            arow = arow_next;
        }
        // the wave's own region: its LDS operations complete in order
        if (c + 1 < nch) st.store_next(c + 1, vb, ubufs, lane);
    }
}

// ---------------------------------------------------------------------------
// FP4 / FP6 operands: v_mfma_scale_f32_32x32x64_f8f6f4 (scale 1), fp32
// accumulation, twice the int8 rate. Small integer codes are exact in these
// formats (E2M1 holds 0..3, E2M3 holds 0..7); every product and partial sum
// is an integer, exact in fp32 while below 2^24 in magnitude, which bounds
// each wave's m range (the host cuts items accordingly). A tile has NB column
// blocks of 32 lags (S = 32 NB, 1024 NB lags; the epilogue is the int8
// engine's for the same NB); a matrix step takes 64 values of m:
//     A[i][k]   = v[q + T0 + S i + k]            k in [0, 64)
//     B_b[k][j] = u[q + k - j - 32 b]
// With q stepping by 64, B_{b+2}(q) = B_b(q - 64): a step reads one A
// fragment and the 64-code u window B_1(q) | B_0(q) (2W + 1 dwords, split
// with v_alignbit) and reuses the pairs of the NB/2 - 1 previous steps for
// the other blocks. NB = 8 halves the LDS bytes per matrix instruction
// against NB = 4 (wide lag ranges); narrow ranges keep NB = 4. Codes are
// packed W bits each, in the operand layout of the instruction (lane (row or
// column, g) holds k = 32 g .. 32 g + 31, code t at bits W t).

template <int W, int NB>
struct FCfg {
    static constexpr int FMT = W == 4 ? kFmtF4 : kFmtF6;
    static constexpr int S = 32 * NB;              // coarse lag stride (samples)
    static constexpr int LS = NB == 4 ? 7 : 8;
    static constexpr int TLW = 32 * S;             // lags per tile, as MCfg<NB>
    static constexpr int KS = 64;                  // m per matrix step
    static constexpr int NP = S / KS;              // B pairs in use = steps per ring block
    static constexpr int CQ = 32;                  // steps per staged chunk
    static constexpr int CM = KS * CQ;             // m per chunk
    static constexpr int VW = TLW + CM;            // v window of a chunk (samples)
    // ring >= VW: as in the int8 engine, the new samples of chunk c+1 are
    // stored after every read of chunk c and replace samples below (c+1) CM
    static constexpr int R = NB == 4 ? 8192 : 16384;
    static_assert(R >= VW, "ring too small");
    static constexpr int SB = S * W / 8;           // packed bytes of S samples
    static constexpr int PAD = W == 4 ? 16 : 8;    // bytes after every S samples (bank spread)
    static constexpr int BLK = SB + PAD;
    static constexpr int VPH = (R / S) * BLK;
    static constexpr int UOFF = 32 * NB;           // u window starts UOFF samples before the chunk
    static constexpr int UW = CM + UOFF + 128;     // u window (samples)
    static constexpr int UB = UW * W / 8;
    static constexpr int WAVE_LDS = VPH + UB;
    static constexpr int FILL_V = VW / 16;         // 16-sample units
    static constexpr int NEW_V = CM / 16;
    static constexpr int U_UNITS = UW / 16;
    static constexpr int FILL_PER_LANE = (FILL_V + U_UNITS + 63) / 64;
    static constexpr int NEXT_PER_LANE = (NEW_V + U_UNITS + 63) / 64;
    static constexpr int BD = 2 * W + 1;           // dwords of a B_1 | B_0 window
    // the windows of the NP - 1 history steps start at sample UOFF - 63 - 64 (NP - 1)
    // >= 0; the last one read (one step past a full chunk) ends inside the u window
    static_assert(UOFF - 63 - KS * (NP - 1) >= 0, "history windows before the u window");
    static_assert(((W * (UOFF + CM)) >> 5) + BD <= UB / 4, "u window too small");
};

// Per-wave staging of packed codes; the same windows as WaveStager, in
// samples, with S samples per padded block of the v ring. Window starts are
// multiples of 16 samples, so every 16-sample unit of a window is one unit of
// the signal's packed array (or lies outside the signal: zeros).
template <int W, int NB>
struct FpStager {
    using C = FCfg<W, NB>;
    Packed16<W> reg[C::NEXT_PER_LANE];
    const uint32_t* upk;     // the descriptor fields, read once (as in WaveStager)
    const uint32_t* vpk;
    int64_t nu, nv;
    __device__ __forceinline__ explicit FpStager(const XPair& p) : upk(p.upk), vpk(p.vpk), nu(p.nu), nv(p.nv) {}

    __device__ __forceinline__ static int vphys(int p) { return (p >> C::LS) * C::BLK + ((p & (C::S - 1)) * W) / 8; }
    __device__ __forceinline__ static void put(uint8_t* dst, const Packed16<W>& c) {
        uint32_t* d = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
        for (int k = 0; k < W / 2; ++k) d[k] = c.d[k];
    }

    __device__ __forceinline__ void fill(int64_t T0, int64_t qw, uint8_t* vb, uint8_t* ub, int lane) {
        lane = opaque(lane);
        const int64_t gv0 = (qw + T0) / 16;            // exact: multiples of 16 (see the host planner)
        const int64_t gu0 = (qw - C::UOFF) / 16;
        Packed16<W> x[C::FILL_PER_LANE];
#pragma unroll
        for (int k = 0; k < C::FILL_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::FILL_V)
                x[k] = load_unit<W>(vpk, nv, gv0 + unit);
            else if (unit < C::FILL_V + C::U_UNITS)
                x[k] = load_unit<W>(upk, nu, gu0 + (unit - C::FILL_V));
        }
#pragma unroll
        for (int k = 0; k < C::FILL_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::FILL_V)
                put(vb + vphys(16 * unit), x[k]);
            else if (unit < C::FILL_V + C::U_UNITS)
                put(ub + 2 * W * (unit - C::FILL_V), x[k]);
        }
    }
    __device__ __forceinline__ void load_next(int64_t T0, int64_t qw, int c, int lane) {
        lane = opaque(lane);
        const int64_t rel0 = (int64_t)(c - 1) * C::CM + C::VW;    // first new window sample
        const int64_t gv0 = (qw + T0 + rel0) / 16;
        const int64_t gu0 = (qw + (int64_t)c * C::CM - C::UOFF) / 16;
#pragma unroll
        for (int k = 0; k < C::NEXT_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::NEW_V)
                reg[k] = load_unit<W>(vpk, nv, gv0 + unit);
            else if (unit < C::NEW_V + C::U_UNITS)
                reg[k] = load_unit<W>(upk, nu, gu0 + (unit - C::NEW_V));
        }
    }
    __device__ __forceinline__ void store_next(int c, uint8_t* vb, uint8_t* ub, int lane) {
        lane = opaque(lane);
        const int rel0 = (int)(((int64_t)(c - 1) * C::CM + C::VW) & (C::R - 1));
#pragma unroll
        for (int k = 0; k < C::NEXT_PER_LANE; ++k) {
            const int unit = lane + 64 * k;
            if (unit < C::NEW_V)
                put(vb + vphys((rel0 + 16 * unit) & (C::R - 1)), reg[k]);
            else if (unit < C::NEW_V + C::U_UNITS)
                put(ub + 2 * W * (unit - C::NEW_V), reg[k]);
        }
    }
};

// int8 codes -> packed units, one thread per unit.
template <int W>
__global__ void __launch_bounds__(256) k_pack_fp(const int8_t* q, int64_t n, uint32_t* pk) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (16 * g >= n) return;
    const Packed16<W> c = fp_pack16<W>(load16_guarded(q, n, 16 * g));
#pragma unroll
    for (int k = 0; k < W / 2; ++k) pk[(W / 2) * g + k] = c.d[k];
}

// The m loop of one wave over [qw_a, qw_b) (a multiple of 64 NP) for the tile
// at T0, FP operands; the partial sums come back as int32.
template <int W, int NB>
__device__ __forceinline__ void wave_loop_fp(const XPair& p, int64_t T0, int64_t qw_a, int64_t qw_b, uint8_t* wl,
                                             int lane, v16i* acc_out, NextItem& nx) {
    using C = FCfg<W, NB>;
    constexpr int NP = C::NP;
    lane = opaque(lane);
    const int lc = lane & 31;
    const int g = lane >> 5;
    uint8_t* vb = wl;
    uint8_t* ub = wl + C::VPH;
    FpStager<W, NB> st(p);
    const int nch = (int)((qw_b - qw_a + C::CM - 1) / C::CM);
    st.fill(T0, qw_a, vb, ub, lane);

    const int brel = C::UOFF + 32 * g - lc - 32;   // first code of the step-0 window
    const uint32_t* ubw = reinterpret_cast<const uint32_t*>(ub) + ((W * brel) >> 5);
    const uint32_t bsh = (uint32_t)((W * brel) & 31);
    const int a_in = (32 * g * W) / 8;             // the lane's k half inside a row
    constexpr int ASTEP = C::KS * W / 8;           // bytes per step along a row

    v16f acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[b][e] = 0.f;

    // The B_1 | B_0 pair of step s sits in slot s mod NP; blocks 2 k and
    // 2 k + 1 take the pair of step s - k. The slots of the steps before the
    // first are read from the history windows. Chunks are whole groups of NP
    // steps, so at a chunk boundary the registers already hold the next
    // chunk's history and its step 0 (read, one step past the old chunk, from
    // staged data that is still valid): only the first chunk reads them.
    v8i hb0[NP], hb1[NP];
#pragma unroll
    for (int k = 1; k < NP; ++k) split_bwin<W>(read_bwin<W>(ubw - 2 * W * k), bsh, hb1[NP - k], hb0[NP - k]);
    // Software pipeline as in the int8 loop: fragments of step s+1 are read
    // while the matrix instructions of step s run (reading one step past the
    // chunk stays inside the staged windows). The NP steps of a group share
    // one padded row block of the ring, so their offsets are constants.
    int blk = ((C::S * lc) & (C::R - 1)) >> C::LS;
    const uint8_t* arow = vb + blk * C::BLK + a_in;
    v8i a_cur = read_a_fp<W>(arow);
    split_bwin<W>(read_bwin<W>(ubw), bsh, hb1[0], hb0[0]);

    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) st.load_next(T0, qw_a, c + 1, lane);
        else nx.fetch();
        const int64_t rem = (qw_b - qw_a - (int64_t)c * C::CM) / C::KS;
        const int nsteps = rem < C::CQ ? (int)rem : C::CQ;
        for (int s0 = 0; s0 < nsteps; s0 += NP) {
            const int nb = (blk + 1) & (C::R / C::S - 1);
            const uint8_t* arow_next = vb + nb * C::BLK + a_in;
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                const int s = s0 + t;
                const v8i a_nxt = read_a_fp<W>(t + 1 < NP ? arow + ASTEP * (t + 1) : arow_next);
                const BWin<W> raw = read_bwin<W>(ubw + 2 * W * (s + 1));
                // FP4 and the 8-block tiles keep the pinned order; the 4-block
                // FP6 loop (wider windows) runs about 5% faster when the
                // compiler interleaves freely
                if (W == 4 || NB == 8) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const int slot = (t - k + NP) % NP;
                    acc[2 * k] = mfma_fp<W>(a_cur, hb0[slot], acc[2 * k]);
                    acc[2 * k + 1] = mfma_fp<W>(a_cur, hb1[slot], acc[2 * k + 1]);
                }
                if (W == 4 || NB == 8) __builtin_amdgcn_sched_barrier(0);
                a_cur = a_nxt;
                // step s + 1 replaces step s + 1 - NP, whose last use was above
                split_bwin<W>(raw, bsh, hb1[(t + 1) % NP], hb0[(t + 1) % NP]);
                if (W == 4 || NB == 8) __builtin_amdgcn_sched_barrier(0);
            }
            blk = nb;
            arow = arow_next;
        }
        if (c + 1 < nch) st.store_next(c + 1, vb, ub, lane);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc_out[b][e] = (int)acc[b][e];
}

// One work item: the wave loops (int8 or FP operands) and the tile's epilogue
// for a tile of MB column blocks.
template <int MB, bool FP>
__device__ __forceinline__ void mfma_tile(const XItem& it, const MWork& wk, uint8_t* lds, ArgPart* tile_parts,
                                          int* counter, int* s_next, void* rbuf) {
    using C = MCfg<MB>;
    const XPair& p = it.p;
    const int64_t T0 = it.T_start + (int64_t)wk.tile * C::TLW;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;

    // quarter of the m range of this item for this wave
    const int64_t part = round_up(ceil_div(wk.qb - wk.qa, 4), 32 * MB);
    const int64_t qw_a = wk.qa + (int64_t)w * part;
    const int64_t qw_b = qw_a + part < wk.qb ? qw_a + part : wk.qb;

    v16i acc[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[b][e] = 0;
    NextItem nx{counter, threadIdx.x == 0, 0};
    if (qw_a < qw_b) {
        if constexpr (FP) {
            if (it.fmt == kFmtF6)
                wave_loop_fp<6, MB>(p, T0, qw_a, qw_b, lds + w * FCfg<6, MB>::WAVE_LDS, lane, acc, nx);
            else
                wave_loop_fp<4, MB>(p, T0, qw_a, qw_b, lds + w * FCfg<4, MB>::WAVE_LDS, lane, acc, nx);
        } else {
            wave_loop<MB>(p, T0, qw_a, qw_b, lds + w * C::WAVE_LDS, lane, acc, nx);
        }
    }
    nx.fetch();                          // the asking lane had no chunk
    if (threadIdx.x == 0) *s_next = nx.v;

    __syncthreads();
    // an FP item's sum is below 4 (2^24 - 1) in magnitude (each wave's cap),
    // so its tile always meets in int32, also inside a wide segmented pair
    const bool wide = !FP && it.wide != 0;
    if (!wide) {
        // ---- int32 tile: the four partials meet by LDS atomics, then every
        // thread takes 16 lags; the argmax triple is kept in 32-bit (tile-
        // local lag k, value, count) and widened once per tile.
        uint32_t* red = reinterpret_cast<uint32_t*>(lds);
        {
            // wave 0 stores its partial (every lag of the tile once), the
            // other waves then add theirs
            const int lc = lane & 31, g = lane >> 5;
            if (w == 0) {
#pragma unroll
                for (int b = 0; b < MB; ++b)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        // accumulator layout: lane (j = lc, g), register e -> row 8(e/4) + 4g + e%4
                        const int i = 8 * (e >> 2) + 4 * g + (e & 3);
                        red[lc + 32 * b + C::S * i] = (uint32_t)acc[b][e];
                    }
            }
            __syncthreads();
            if (w != 0) {
#pragma unroll
                for (int b = 0; b < MB; ++b)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int i = 8 * (e >> 2) + 4 * g + (e & 3);
                        // unconditional: a test per value costs more in
                        // branches than the adds it would skip
                        atomicAdd(red + lc + 32 * b + C::S * i, (unsigned int)acc[b][e]);
                    }
            }
        }
        __syncthreads();
        // the pair's fields, read once: the r stores below go through generic
        // pointers and would make the compiler re-read them per lag
        void* const r = rbuf;
        const int r_dtype = p.r_dtype;
        const bool segmented = wk.segmented != 0;
        const int64_t lag_lo = p.lag_lo;
        // lags of the tile inside [lag_lo, lag_hi]: k in [klo, khi]
        const int64_t klo64 = lag_lo - T0, khi64 = p.lag_hi - T0;
        const int klo = klo64 < 0 ? 0 : (int)klo64;
        const int khi = khi64 >= C::TLW ? C::TLW - 1 : (int)khi64;
        // thread t takes lags 1024 j + 4 t + e, four per LDS read, the read of
        // the next four issued before the current ones are used
        constexpr int NJ = C::TLW / 1024;
        uint4 cur = *reinterpret_cast<const uint4*>(red + 4 * threadIdx.x);
        int bv = INT32_MIN, bk = INT32_MAX, bc = 0;
#pragma unroll 1
        for (int j = 0; j < NJ; ++j) {
            const uint4 nxt = *reinterpret_cast<const uint4*>(red + 1024 * ((j + 1) % NJ) + 4 * threadIdx.x);
            const uint32_t q4[4] = {cur.x, cur.y, cur.z, cur.w};
            cur = nxt;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 1024 * j + 4 * (int)threadIdx.x + e;
                if (k < klo || k > khi) continue;
                const int v = (int)q4[e];
                if (r) {
                    const int64_t idx = T0 + k - lag_lo;
                    if (segmented) {
                        if (v != 0) {
                            if (r_dtype == TDE_I32)
                                atomicAdd(static_cast<int*>(r) + idx, v);
                            else
                                atomicAdd(static_cast<unsigned long long*>(r) + idx, (unsigned long long)(long long)v);
                        }
                    } else if (r_dtype == TDE_I32) {
                        static_cast<int32_t*>(r)[idx] = v;
                    } else {
                        static_cast<int64_t*>(r)[idx] = v;
                    }
                }
                // k increases along the thread's lags: a new maximum resets, an equal one counts
                if (v > bv) {
                    bv = v;
                    bk = k;
                    bc = 1;
                } else if (v == bv) {
                    bc += 1;
                }
            }
        }
        if (tile_parts && !wk.segmented) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int ov = __shfl_xor(bv, o, 64), ok = __shfl_xor(bk, o, 64), oc = __shfl_xor(bc, o, 64);
                if (ov > bv) {
                    bv = ov;
                    bk = ok;
                    bc = oc;
                } else if (ov == bv) {
                    bk = ok < bk ? ok : bk;
                    bc += oc;
                }
            }
            __shared__ int sh32[4][3];
            if (lane == 0) {
                sh32[w][0] = bv;
                sh32[w][1] = bk;
                sh32[w][2] = bc;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                Tri64 a{INT64_MIN, INT64_MAX, 0};
                for (int q = 0; q < 4; ++q)
                    if (sh32[q][2] > 0) a = tri_join(a, Tri64{sh32[q][0], T0 + sh32[q][1] - p.lag_lo, sh32[q][2]});
                tile_parts[it.part_base + wk.tile] = ArgPart{a.v, a.i, a.c};
            }
        }
        return;
    }
    // ---- int64 tile (sums may exceed int32): partials meet by LDS atomics
    if (wide) {
        unsigned long long* red = reinterpret_cast<unsigned long long*>(lds);
        for (int k = threadIdx.x; k < C::TLW; k += 256) red[k] = 0ull;
    } else {
        uint32_t* red = reinterpret_cast<uint32_t*>(lds);
        for (int k = threadIdx.x; k < C::TLW; k += 256) red[k] = 0u;
    }
    __syncthreads();
    {
        // accumulator layout: lane (j = lc, g), register e -> row 8(e/4) + 4g + e%4
        const int lc = lane & 31, g = lane >> 5;
        if (wide) {
#pragma unroll
            for (int b = 0; b < MB; ++b)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    atomicAdd(reinterpret_cast<unsigned long long*>(lds) + lc + 32 * b + C::S * (8 * (e >> 2) + 4 * g + (e & 3)),
                              (unsigned long long)(long long)acc[b][e]);
        } else {
#pragma unroll
            for (int b = 0; b < MB; ++b)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    atomicAdd(reinterpret_cast<unsigned int*>(lds) + lc + 32 * b + C::S * (8 * (e >> 2) + 4 * g + (e & 3)),
                              (unsigned int)acc[b][e]);
        }
    }
    __syncthreads();

    // ---- outputs: r (plain stores or, for segments, atomics) and the triple
    void* const r = rbuf;                // read once (as in the int32 path)
    const int r_dtype = p.r_dtype;
    const bool segmented = wk.segmented != 0;
    const int64_t lag_lo = p.lag_lo;
    const int64_t L = p.lag_hi - lag_lo + 1;
    Tri64 t{INT64_MIN, INT64_MAX, 0};
    for (int k = threadIdx.x; k < C::TLW; k += 256) {
        const int64_t tau = T0 + k;
        const int64_t idx = tau - lag_lo;
        if (idx < 0 || idx >= L) continue;
        const int64_t val = wide ? (int64_t)reinterpret_cast<const unsigned long long*>(lds)[k]
                                 : (int64_t)(int32_t)reinterpret_cast<const uint32_t*>(lds)[k];
        if (r) {
            if (segmented) {
                if (val != 0) {
                    if (r_dtype == TDE_I32)
                        atomicAdd(static_cast<int*>(r) + idx, (int)val);
                    else
                        atomicAdd(static_cast<unsigned long long*>(r) + idx, (unsigned long long)val);
                }
            } else if (r_dtype == TDE_I32) {
                static_cast<int32_t*>(r)[idx] = (int32_t)val;
            } else {
                static_cast<int64_t*>(r)[idx] = val;
            }
        }
        t = tri_join(t, Tri64{val, idx, 1});
    }
    if (tile_parts && !wk.segmented) {
        // workgroup reduction of the triple
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            Tri64 u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
            t = tri_join(t, u);
        }
        __shared__ Tri64 sh[4];
        if (lane == 0) sh[w] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            Tri64 a = tri_join(tri_join(sh[0], sh[1]), tri_join(sh[2], sh[3]));
            tile_parts[it.part_base + wk.tile] = ArgPart{a.v, a.i, a.c};
        }
    }
}

// Persistent: each workgroup takes items until the list is exhausted; every
// wave of the grid reaches the exit once the counter passes nwork.
// A value written by an earlier kernel of the same call, read with a
// device-scope load (not through the scalar cache).
__device__ __forceinline__ uint64_t fresh_u64(const void* p) {
    return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int fresh_int(const int* p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ MWork fresh_work(const MWork* p) {
    constexpr int N = sizeof(MWork) / 8;
    static_assert(sizeof(MWork) % 8 == 0, "whole 8-byte words");
    uint64_t w[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint64_t v = fresh_u64(reinterpret_cast<const uint64_t*>(p) + k);
        w[k] = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)v);
    }
    return __builtin_bit_cast(MWork, w);
}

template <int MB>
__global__ void __launch_bounds__(256, MB == 4 ? 2 : 1) k_xcorr_mfma(const XItem* __restrict__ items,
                                                                      const MWork* __restrict__ work, int nwork,
                                                                      int* counter, ArgPart* tile_parts,
                                                                      const int* nwork_dev, uint8_t* rpool,
                                                                      int64_t slot_bytes) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ int s_item;
    // a list planned on the device (nwork was its capacity): its length and
    // items come through device-scope loads
    if (nwork_dev) nwork = fresh_int(nwork_dev);
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    for (;;) {
        // uniform: descriptors come through scalar loads, not VGPRs
        const int wi = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();                  // every wave has read s_item
        if (wi >= nwork) break;
        const MWork wk = nwork_dev ? fresh_work(work + wi) : work[wi];
        const XItem& it = items[wk.pair];
        void* const rbuf = wk.rslot ? rpool + (int64_t)(wk.rslot - 1) * slot_bytes : it.p.r;
        if (it.margin && *it.margin >= it.theta) {   // learned mode: windows suffice
            if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
            __syncthreads();
            continue;
        }
        // the list holds only items of this variant: FP items (4 or 8 blocks)
        // run in the 4-block launch. Each item leaves the next one in s_item.
        if (MB == 4 && wk.fmt != kFmtI8) {
            if (wk.mb == 8)
                mfma_tile<8, true>(it, wk, lds, tile_parts, counter, &s_item, rbuf);
            else
                mfma_tile<4, true>(it, wk, lds, tile_parts, counter, &s_item, rbuf);
        } else {
            mfma_tile<MB, false>(it, wk, lds, tile_parts, counter, &s_item, rbuf);
        }
        __syncthreads();
    }
}

__global__ void k_zero_counters(int* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// Per pair: join the tile triples with the triple of the lags no tile covers
// (their correlation is 0) and write the peak.
__global__ void __launch_bounds__(64) k_tiles_final(const XItem* items, XItem one, int npairs,
                                                    const ArgPart* tile_parts) {
    (void)npairs;                    // the grid has one workgroup per pair
    const int pi = blockIdx.x;
    const XItem& it = items ? items[pi] : one;
    if (!it.fused) return;
    // learned mode: the proposed windows, unless the pair fell back
    const bool windows = it.margin && *it.margin >= it.theta;
    Tri64 t{INT64_MIN, INT64_MAX, 0};
    if (windows) {
        for (int k = threadIdx.x; k < it.nwin; k += 64) {
            ArgPart a = it.win_parts[k];
            t = tri_join(t, Tri64{a.vmax, a.idx, a.cnt});
        }
    } else {
        if (threadIdx.x == 0) t = Tri64{it.out_v, it.out_i, it.out_c};
        for (int64_t k = threadIdx.x; k < it.ntiles; k += 64) {
            ArgPart a = tile_parts[it.part_base + k];
            t = tri_join(t, Tri64{a.vmax, a.idx, a.cnt});
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Tri64 u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
        t = tri_join(t, u);
    }
    if (threadIdx.x == 0) {
        const int flags = peak_flags(it.stat_x, it.p.nu, it.stat_y, it.p.nv) |
                          (it.margin && !windows ? TDE_FLAG_FALLBACK : 0);
        tde_peak pk;
        pk.lag = it.p.lag_lo + t.i;
        pk.rmax = t.v;
        pk.n_ties = (int32_t)t.c;
        pk.flags = flags;
        *it.peak = pk;
    }
}

// ----------------------------------------------------------------- host --

static void clamp_support(const XPair& p, int64_t& lo, int64_t& hi) {
    lo = p.lag_lo > -(p.nu - 1) ? p.lag_lo : -(p.nu - 1);
    hi = p.lag_hi < p.nv - 1 ? p.lag_hi : p.nv - 1;
}

// m range [Q_lo, Q_lo + len) of the tile starting at T0 (len a multiple of
// 4 waves x MB steps x 32).
template <int MB>
static void tile_range(const XPair& p, int64_t T0, int64_t& Q_lo, int64_t& len) {
    using C = MCfg<MB>;
    const int64_t T1 = T0 + C::TLW - 1;
    const int64_t m_lo = T1 < 0 ? -T1 : 0;
    const int64_t m_hi = p.nu < p.nv - T0 ? p.nu : p.nv - T0;
    if (m_hi <= m_lo) {
        Q_lo = 0;
        len = 0;
        return;
    }
    Q_lo = (m_lo / 32) * 32;
    len = round_up(m_hi + C::S - Q_lo, 4 * 32 * MB);
}

static void tile_range_mb(const XItem& it, int64_t t, int64_t& Q_lo, int64_t& len) {
    if (it.mb == 8) tile_range<8>(it.p, it.T_start + t * MCfg<8>::TLW, Q_lo, len);
    else tile_range<4>(it.p, it.T_start + t * MCfg<4>::TLW, Q_lo, len);
}

// Longest m range one item may cover: each wave's quarter stays exact in its
// accumulators (int32, or fp32 integers below 2^24 for FP operands).
static int64_t seg_cap(const XItem& it) {
    const int64_t unit = 32 * (int64_t)it.mb;
    const int64_t lim = it.fmt == kFmtI8 ? (int64_t)0x7fffffff : ((int64_t)1 << 24) - 1;
    const int64_t per_wave = (lim / it.p.kuv) / unit * unit;
    return 4 * per_wave;
}

// FP4 for codes up to 3, FP6 up to 7 (both exact), int8 beyond.
int mfma_choose_fmt(int kmax, bool allow_fp) {
    if (!allow_fp || kmax < 1) return kFmtI8;
    if (kmax <= 3) return kFmtF4;
    if (kmax <= 7) return kFmtF6;
    return kFmtI8;
}

// Lags of [lo, hi] (the clamped range) covered by tiles of tlw lags.
static int64_t tiled_lags(int64_t lo, int64_t hi, int64_t tlw) {
    const int64_t L = hi - floor_div(lo, 16) * 16 + 1;
    return ceil_div(L, tlw) * tlw;
}

// int8 items: 4 accumulator blocks (4096-lag tiles) unless the tuning table
// picked 8 for the pair's bucket (the separate 8-block launch, one wave per
// SIMD).
int choose_mb(const XPair& p) {
    return tuned_tile_blocks(p.nu, p.nv, p.kuv, p.lag_lo, p.lag_hi) == 8 ? 8 : 4;
}

// FP tiles: the tuning table's choice for the pair's bucket; without one,
// 8 blocks (8192 lags) unless that computes more than 1/8 more lags than
// 4-block tiles would, or the shorter signal has fewer than 32768 samples:
// then each wave's share of a tile is a few chunks, fixed per-item costs
// dominate, and twice as many 4-block items spread over more workgroups.
static int choose_fp_nb(const XPair& p) {
    const int tuned = tuned_tile_blocks(p.nu, p.nv, p.kuv, p.lag_lo, p.lag_hi);
    if (tuned == 4 || tuned == 8) return tuned;
    if ((p.nu < p.nv ? p.nu : p.nv) < 32768) return 4;
    int64_t lo, hi;
    clamp_support(p, lo, hi);
    if (lo > hi) return 4;
    return 8 * tiled_lags(lo, hi, MCfg<8>::TLW) <= 9 * tiled_lags(lo, hi, MCfg<4>::TLW) ? 8 : 4;
}

void mfma_plan_pair(XItem& it, bool allow_fp) {
    it.fmt = mfma_choose_fmt(it.p.kmax, allow_fp);
    it.mb = it.fmt == kFmtI8 ? choose_mb(it.p) : choose_fp_nb(it.p);
    const int64_t TLW = it.mb == 8 ? MCfg<8>::TLW : MCfg<4>::TLW;
    int64_t lo, hi;
    clamp_support(it.p, lo, hi);
    it.ntiles = 0;
    it.T_start = 0;
    it.segmented = 0;
    it.wide = 0;
    if (lo <= hi) {
        it.T_start = floor_div(lo, 16) * 16;
        it.ntiles = ceil_div(hi - it.T_start + 1, TLW);
    }
    int64_t maxlen = 0;
    for (int64_t t = 0; t < it.ntiles; ++t) {
        int64_t Q_lo, len;
        tile_range_mb(it, t, Q_lo, len);
        if (len > maxlen) maxlen = len;
    }
    if (maxlen > seg_cap(it)) it.segmented = 1;
    // a tile sum can exceed int32 only if its m range times Ku Kv does
    if ((__int128)maxlen * it.p.kuv >= ((__int128)1 << 31)) it.wide = 1;
    // lags of [lag_lo, lag_hi] outside every tile: r = 0 there
    const int64_t L = it.p.lag_hi - it.p.lag_lo + 1;
    int64_t c_lo = it.T_start, c_hi = it.T_start + it.ntiles * TLW - 1;   // covered lags
    if (it.ntiles == 0) {
        c_lo = 1;
        c_hi = 0;
    }
    c_lo = c_lo > it.p.lag_lo ? c_lo : it.p.lag_lo;
    c_hi = c_hi < it.p.lag_hi ? c_hi : it.p.lag_hi;
    const int64_t covered = c_hi >= c_lo ? c_hi - c_lo + 1 : 0;
    it.out_c = L - covered;
    if (it.out_c == 0) {
        it.out_v = INT64_MIN;
        it.out_i = INT64_MAX;
    } else {
        it.out_v = 0;
        it.out_i = (covered == 0 || c_lo > it.p.lag_lo) ? 0 : (c_hi + 1 - it.p.lag_lo);
    }
}

int64_t mfma_total_q(const XItem& it) {
    int64_t tot = 0;
    for (int64_t t = 0; t < it.ntiles; ++t) {
        int64_t Q_lo, len;
        tile_range_mb(it, t, Q_lo, len);
        tot += len;
    }
    return tot;
}

int64_t mfma_count_items(const XItem& it) {
    const int64_t cap = seg_cap(it);
    int64_t n = 0;
    for (int64_t t = 0; t < it.ntiles; ++t) {
        int64_t Q_lo, len;
        tile_range_mb(it, t, Q_lo, len);
        n += len == 0 ? 1 : ceil_div(len, cap);
    }
    return n;
}

void mfma_items(const XItem& it, int pair, std::vector<MWork>& out) {
    const int64_t cap = seg_cap(it);
    for (int64_t t = 0; t < it.ntiles; ++t) {
        int64_t Q_lo, len;
        tile_range_mb(it, t, Q_lo, len);
        if (len == 0) {
            // no overlap anywhere in the tile: an empty item writes its zeros
            out.push_back(MWork{pair, (int32_t)t, 0, 0, it.segmented, it.mb, it.fmt, 0});
            continue;
        }
        for (int64_t o = 0; o < len; o += cap)
            out.push_back(MWork{pair, (int32_t)t, Q_lo + o, Q_lo + (o + cap < len ? o + cap : len), it.segmented,
                                it.mb, it.fmt, 0});
    }
}

// Most expensive first (matrix work grows with the m range and the tile's
// blocks; an FP instruction covers twice the m of an int8 one), the items of
// the 4-block launch ahead of the 8-block int8 ones (two launches).
static int64_t item_cost(const MWork& a) { return (a.qb - a.qa) * a.mb * (a.fmt == kFmtI8 ? 2 : 1); }

void mfma_sort_items(std::vector<MWork>& w) {
    std::stable_sort(w.begin(), w.end(), [](const MWork& a, const MWork& b) {
        const int ka = mfma_launch_of(a.fmt, a.mb), kb = mfma_launch_of(b.fmt, b.mb);
        if (ka != kb) return ka < kb;
        return item_cost(a) > item_cost(b);
    });
}

// Dynamic LDS of a launch: the 4-block launch also runs the FP items.
template <int MB>
constexpr int kernel_lds() {
    if (MB == 8) return MCfg<8>::LDS;
    int l = MCfg<4>::LDS;
    const int f[4] = {4 * FCfg<6, 4>::WAVE_LDS, 4 * FCfg<4, 4>::WAVE_LDS, 4 * FCfg<6, 8>::WAVE_LDS,
                      4 * FCfg<4, 8>::WAVE_LDS};
    for (int k = 0; k < 4; ++k) l = f[k] > l ? f[k] : l;
    return l;
}
// the int32 epilogue of an 8-block FP tile meets in the 4-block launch's LDS
static_assert(kernel_lds<4>() >= MCfg<8>::TLW * 4, "FP 8-block reduction area");

template <int MB>
static int launch_mb(const XItem* items_dev, const MWork* work, int nwork, int* counter, ArgPart* tile_parts,
                     int num_cu, hipStream_t s, const int* nwork_dev, uint8_t* rpool, int64_t slot_bytes) {
    if (nwork == 0) return TDE_OK;
    static int per_cu = 0;
    if (per_cu == 0) {
        TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_xcorr_mfma<MB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          kernel_lds<MB>()));
        int nb = 0;
        TDE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_xcorr_mfma<MB>, 256, kernel_lds<MB>()));
        per_cu = nb > 0 ? nb : 1;
    }
    int grid = per_cu * num_cu;
    if (grid > nwork) grid = nwork;
    hipLaunchKernelGGL(k_xcorr_mfma<MB>, dim3(grid), dim3(256), kernel_lds<MB>(), s, items_dev, work, nwork, counter,
                       tile_parts, nwork_dev, rpool, slot_bytes);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_xcorr_mfma(const XItem* items_dev, const MWork* work_dev, int nwork, int* counters_dev,
                      bool counters_zeroed, ArgPart* tile_parts, int num_cu, hipStream_t s, int n4,
                      const int* nwork_dev, uint8_t* rpool, int64_t slot_bytes) {
    if (!counters_zeroed) {
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, counters_dev, 2);
        TDE_HIP_CHECK(hipGetLastError());
    }
    // a device-planned list holds 4-block-launch items only
    int rc = launch_mb<4>(items_dev, work_dev, n4, counters_dev, tile_parts, num_cu, s, nwork_dev, rpool, slot_bytes);
    if (rc) return rc;
    if (nwork_dev) return TDE_OK;
    return launch_mb<8>(items_dev, work_dev + n4, nwork - n4, counters_dev + 1, tile_parts, num_cu, s, nullptr,
                        nullptr, 0);
}

int launch_pack_fp(const int8_t* q, int64_t n, uint32_t* pk, int W, hipStream_t s) {
    const int64_t units = (n + 15) / 16;
    if (units == 0) return TDE_OK;
    const unsigned blocks = (unsigned)((units + 255) / 256);
    if (W == 6)
        hipLaunchKernelGGL(k_pack_fp<6>, dim3(blocks), dim3(256), 0, s, q, n, pk);
    else
        hipLaunchKernelGGL(k_pack_fp<4>, dim3(blocks), dim3(256), 0, s, q, n, pk);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_tiles_final(const XItem* items_dev, const XItem& one, int npairs, const ArgPart* tile_parts,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_tiles_final, dim3(npairs), dim3(64), 0, s, items_dev, one, npairs, tile_parts);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

// ------------------------------------------- learned fallback, on device --
// One workgroup: the pairs below the margin threshold (in pair order), their
// items, and the split factor S that makes about `target` items; then the
// work list, and for S > 1 the pairs' r slots. ctl[0]: pairs with a slot
// (0 when S <= 1), ctl[1]: items in the list.
__global__ void __launch_bounds__(1024) k_fb_plan(const XItem* items, int npairs, const MWork* __restrict__ swork,
                                                  MWork* dwork, int* ctl, int* slots, int target) {
    __shared__ int s_sum[2][32];
    __shared__ int s_tot[2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto falls = [&](int i) { return !(*items[i].margin >= items[i].theta); };
    // pass 1: how many pairs fall back, and their items
    int nf = 0, ni = 0;
    for (int i = tid; i < npairs; i += 1024)
        if (falls(i)) {
            nf += 1;
            ni += items[i].work_count;
        }
    for (int o = 32; o > 0; o >>= 1) {
        nf += __shfl_xor(nf, o, 64);
        ni += __shfl_xor(ni, o, 64);
    }
    if (lane == 0) {
        s_sum[0][wv] = nf;
        s_sum[1][wv] = ni;
    }
    __syncthreads();
    if (tid == 0) {
        int a = 0, b = 0;
        for (int k = 0; k < 16; ++k) {
            a += s_sum[0][k];
            b += s_sum[1][k];
        }
        s_tot[0] = a;
        s_tot[1] = b;
    }
    __syncthreads();
    const int NF = s_tot[0], NI = s_tot[1];
    int S = 1;
    if (NF > 0 && NF <= kFbSlots && NI < target) {
        S = (target + NI - 1) / NI;
        S = S > kFbMaxSplit ? kFbMaxSplit : S;
    }
    // pass 2: the list, chunk by chunk of 1024 pairs. Exclusive scans of the
    // item counts and of the fallback flags give each fallback pair of the
    // chunk its first list position and its slot; then every thread writes
    // list entries, finding an entry's pair by binary search over the
    // chunk's first positions.
    __shared__ int s_fpair[1024], s_fstart[1024];
    int base_items = 0, base_slot = 0;
    for (int c0 = 0; c0 < npairs; c0 += 1024) {
        __syncthreads();
        const int i = c0 + tid;
        const bool fb = i < npairs && falls(i);
        const int cnt = fb ? items[i].work_count * S : 0, one = fb ? 1 : 0;
        int pc = cnt, po = one;                       // inclusive scans inside the wave
        for (int o = 1; o < 64; o <<= 1) {
            const int a = __shfl_up(pc, o, 64), b = __shfl_up(po, o, 64);
            if (lane >= o) {
                pc += a;
                po += b;
            }
        }
        if (lane == 63) {
            s_sum[0][wv] = pc;
            s_sum[1][wv] = po;
        }
        __syncthreads();
        int wc = 0, wo = 0, tc = 0, to = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < wv) {
                wc += s_sum[0][k];
                wo += s_sum[1][k];
            }
            tc += s_sum[0][k];
            to += s_sum[1][k];
        }
        if (fb) {
            const int ci = wo + po - one;
            s_fpair[ci] = i;
            s_fstart[ci] = wc + pc - cnt;
            if (S > 1) slots[base_slot + ci] = i;
        }
        __syncthreads();
        for (int o = tid; o < tc; o += 1024) {
            // the last fallback pair of the chunk whose first position is <= o
            // (pairs without items share their successor's first position)
            int lo = 0, hi = to - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_fstart[mid] <= o) lo = mid;
                else hi = mid - 1;
            }
            const int rel = o - s_fstart[lo], j = rel / S, k = rel - j * S;
            const MWork w = swork[items[s_fpair[lo]].work_first + j];
            if (S == 1) {
                dwork[base_items + o] = w;
                continue;
            }
            // segments of whole 4 x 32 mb steps (the cut of a long tile)
            const int64_t unit = 128 * (int64_t)w.mb, len = w.qb - w.qa;
            const int64_t seg = (len + S - 1) / S;
            const int64_t step = (seg + unit - 1) / unit * unit;
            MWork x = w;
            const int64_t a = w.qa + k * step;
            x.qa = a < w.qb ? a : w.qb;
            x.qb = a + step < w.qb ? a + step : w.qb;
            x.segmented = 1;
            x.rslot = base_slot + lo + 1;
            dwork[base_items + o] = x;
        }
        base_items += tc;
        base_slot += to;
    }
    if (tid == 0) {
        ctl[0] = S > 1 ? NF : 0;
        ctl[1] = NI * S;
    }
}

// grid (kFbSlots, 64): the r slots of the split pairs to zero.
__global__ void __launch_bounds__(256) k_fb_zero(const XItem* items, const int* ctl, const int* slots,
                                                 uint8_t* rpool, int64_t slot_bytes) {
    const int k = blockIdx.x;
    if (k >= fresh_int(ctl)) return;
    const XPair& p = items[fresh_int(slots + k)].p;
    const int64_t bytes = (p.lag_hi - p.lag_lo + 1) * (p.r_dtype == TDE_I32 ? 4 : 8);
    uint8_t* r = rpool + (int64_t)k * slot_bytes;     // 16-byte aligned slot, whole 16-byte pieces
    for (int64_t e = 16 * ((int64_t)blockIdx.y * 256 + threadIdx.x); e < bytes; e += 16 * 256 * 64)
        *reinterpret_cast<uint4*>(r + e) = make_uint4(0u, 0u, 0u, 0u);
}

// grid (kFbSlots, kFbChunks): (max, first lag, count) of a split pair's r
// over one of kFbChunks consecutive parts of its lags (lags no tile covers
// kept their zero), four values per load.
constexpr int kFbChunks = 64;
__global__ void __launch_bounds__(256) k_fb_argmax_parts(const XItem* items, const int* ctl, const int* slots,
                                                         const uint8_t* rpool, int64_t slot_bytes, ArgPart* parts) {
    const int k = blockIdx.x, c = blockIdx.y;
    if (k >= fresh_int(ctl)) return;
    const XItem& it = items[fresh_int(slots + k)];
    const int64_t L = it.p.lag_hi - it.p.lag_lo + 1;
    const int64_t per = ((L + kFbChunks - 1) / kFbChunks + 3) / 4 * 4;     // keeps 16-byte loads aligned
    const int64_t lo = c * per, hi = lo + per < L ? lo + per : L;
    const bool i32 = it.p.r_dtype == TDE_I32;
    const uint8_t* r = rpool + (int64_t)k * slot_bytes;
    Tri64 t{INT64_MIN, INT64_MAX, 0};
    for (int64_t e0 = lo + 4 * (int64_t)threadIdx.x; e0 < hi; e0 += 4 * 256) {
        int64_t v[4];
        if (i32 && e0 + 4 <= hi && (e0 & 3) == 0) {
            const int4 q = *reinterpret_cast<const int4*>(r + 4 * e0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[e] = e0 + e >= hi ? INT64_MIN
                       : i32        ? (int64_t) reinterpret_cast<const int32_t*>(r)[e0 + e]
                                    : reinterpret_cast<const int64_t*>(r)[e0 + e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (e0 + e < hi) t = tri_join(t, Tri64{v[e], e0 + e, 1});
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Tri64 u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
        t = tri_join(t, u);
    }
    __shared__ Tri64 sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        t = tri_join(tri_join(sh[0], sh[1]), tri_join(sh[2], sh[3]));
        parts[k * kFbChunks + c] = ArgPart{t.v, t.i, t.c};
    }
}

// grid kFbSlots: the peaks of the split pairs from their parts.
__global__ void __launch_bounds__(64) k_fb_argmax(const XItem* items, const int* ctl, const int* slots,
                                                  const ArgPart* parts) {
    const int k = blockIdx.x;
    if (k >= fresh_int(ctl)) return;
    const XItem& it = items[fresh_int(slots + k)];
    const ArgPart a = parts[k * kFbChunks + threadIdx.x];
    Tri64 t{a.vmax, a.idx, a.cnt};
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Tri64 u{__shfl_xor(t.v, o, 64), __shfl_xor(t.i, o, 64), __shfl_xor(t.c, o, 64)};
        t = tri_join(t, u);
    }
    if (threadIdx.x == 0) {
        tde_peak pk;
        pk.lag = it.p.lag_lo + t.i;
        pk.rmax = t.v;
        pk.n_ties = (int32_t)t.c;
        pk.flags = peak_flags(it.stat_x, it.p.nu, it.stat_y, it.p.nv) | TDE_FLAG_FALLBACK;
        *it.peak = pk;
    }
}
static_assert(kFbChunks == 64, "one part per lane of the final wave");

int launch_fb_plan(const XItem* items_dev, int npairs, const MWork* swork, MWork* dwork, int* ctl, int* slots,
                   int target, hipStream_t s) {
    hipLaunchKernelGGL(k_fb_plan, dim3(1), dim3(1024), 0, s, items_dev, npairs, swork, dwork, ctl, slots, target);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_fb_zero(const XItem* items_dev, const int* ctl, const int* slots, uint8_t* rpool, int64_t slot_bytes,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_fb_zero, dim3(kFbSlots, 64), dim3(256), 0, s, items_dev, ctl, slots, rpool, slot_bytes);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_fb_argmax(const XItem* items_dev, const int* ctl, const int* slots, const uint8_t* rpool,
                     int64_t slot_bytes, ArgPart* parts, hipStream_t s) {
    hipLaunchKernelGGL(k_fb_argmax_parts, dim3(kFbSlots, kFbChunks), dim3(256), 0, s, items_dev, ctl, slots, rpool,
                       slot_bytes, parts);
    TDE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_fb_argmax, dim3(kFbSlots), dim3(64), 0, s, items_dev, ctl, slots, parts);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

}  // namespace tde
