// Learned lag-window proposer (not part of the paper): a small 1-D CNN over
// decimated signals whose feature cross-correlation scores coarse lag bins,
// so that the exact integer correlation (Algorithm 1, correlation step) is evaluated
// only inside the best bins.
//
//   input   xd[t] = bf16(mean of x[16t .. 16t+15] / sigma), t < Ld
//   layer l (4 of them, C = 32 channels, kernel 9, zero padding 4):
//           Z[t][o] = b[o] + sum_i sum_k W[o][i][k] X[t + k - 4][i]
//           P[t][o] = (relu(Z[2t][o]) + relu(Z[2t+1][o])) / 2      (next X)
//   head    raw[k] = sum_t sum_c Fx[t][c] Fy[t + k - nb/2][c],  logits = alpha raw
//
// Storage: activations bf16, position-major ([t][c], 64 bytes per position);
// arithmetic fp32. The weights and biases used by the kernels are
// bf16-rounded copies of fp32 master weights (kept as float); alpha stays
// float32. Training: softmax cross-entropy,
// backward through head, pooling, ReLU and convolutions, Adam on the masters.
// Signals are indexed g = 2 * pair + side (side 0: x, 1: y).
#include "tde_internal.h"

namespace tde {

namespace {

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);     // round to nearest even
}

}  // namespace

__device__ __forceinline__ float bf16_round_dev(float f) { return bf2f(f2bf(f)); }

// ------------------------------------------------------------- decimate --
// out[g][t] = bf16(mean16(x_g) * scale_g); one thread per output sample.
__global__ void __launch_bounds__(256) k_cnn_decimate(const CnnSig* sigs, int ld, uint16_t* out) {
    const int g = blockIdx.y;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= ld) return;
    const CnnSig s = sigs[g];
    const float* x = s.x + (int64_t)16 * t;
    // ((x0+x1)+(x2+x3)) per quad, then (q0+q1)+(q2+q3): the order of the
    // decimation fused into the quantize kernel
    float q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = (x[4 * k] + x[4 * k + 1]) + (x[4 * k + 2] + x[4 * k + 3]);
    const float acc = (q[0] + q[1]) + (q[2] + q[3]);
    const float scale = s.inv ? (*s.inv) * s.scale_mul : s.scale_mul;
    out[(int64_t)g * ld + t] = f2bf(acc * (1.f / 16.f) * scale);
}

// ---------------------------------------------------------- conv layer 0 --
// One input channel. grid (ceil(L / 512), nsig); thread -> one pooled
// position (two conv positions), all 32 channels. The weights are the same
// for every thread: they come through scalar loads as instruction operands
// (W[c K + k], bias[c]), not through LDS.
template <bool SAVE>
__global__ void __launch_bounds__(256) k_conv1_fwd(const uint16_t* __restrict__ X, const float* __restrict__ W,
                                                   const float* __restrict__ bias, uint16_t* __restrict__ Z,
                                                   uint16_t* __restrict__ P, int L) {
    const int g = blockIdx.y;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (2 * p >= L) return;
    const uint16_t* x = X + (int64_t)g * L;
    float xv[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const int t = 2 * p - 4 + j;
        xv[j] = (t >= 0 && t < L) ? bf2f(x[t]) : 0.f;
    }
    uint16_t zo[2][kCnnC];
    uint16_t po[kCnnC];
#pragma unroll
    for (int c = 0; c < kCnnC; ++c) {
        float z0 = bias[c], z1 = bias[c];
#pragma unroll
        for (int k = 0; k < kCnnK; ++k) {
            z0 += W[c * kCnnK + k] * xv[k];
            z1 += W[c * kCnnK + k] * xv[k + 1];
        }
        zo[0][c] = f2bf(z0);
        zo[1][c] = f2bf(z1);
        po[c] = f2bf(0.5f * (fmaxf(z0, 0.f) + fmaxf(z1, 0.f)));
    }
    if (SAVE) {
        uint4* zd = reinterpret_cast<uint4*>(Z + ((int64_t)g * L + 2 * p) * kCnnC);
#pragma unroll
        for (int q = 0; q < 8; ++q) zd[q] = reinterpret_cast<const uint4*>(&zo[0][0])[q];
    }
    uint4* pd = reinterpret_cast<uint4*>(P + ((int64_t)g * (L / 2) + p) * kCnnC);
#pragma unroll
    for (int q = 0; q < 4; ++q) pd[q] = reinterpret_cast<const uint4*>(po)[q];
}

constexpr int kTile = 128;           // backward-data tile (positions)
constexpr int kXs = kTile + 8;       // input rows with halo

// ------------------------------------------------ conv layers 1+ (MFMA) --
// Implicit GEMM on the bf16 matrix cores (v_mfma_f32_32x32x16_bf16):
//   C[o][t] = sum_kk A[o][kk] B[kk][t],  kk = 32 tap + i,
//   A[o][kk] = W[o][i][tap],  B[kk][t] = X[t + tap - 4][i]
// One matrix instruction per block of 16 kk (fixed tap, 16 channels): 18 per
// 32 x 32 output tile. The weights of a layer sit in registers as 18
// per-lane fragments (packed once per weight update); the B fragment of a
// lane is 8 consecutive channels of one input position, one 16-byte LDS
// read. A workgroup stages 512 + 8 input rows; each wave makes 4 tiles.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMPos = 512;                 // positions per workgroup
constexpr int kMRow = 80;                  // LDS bytes per staged row (64 + pad)

// frag[b][lane] (8 bf16): row o = lane % 32, kk = 16 b + 8 (lane / 32) + j,
// of scale * W (scale 1, or 1/2 for the fused inference kernel: halving a
// bf16 weight is exact)
__global__ void k_pack_wfrag(const float* W, uint4* frag, float scale) {
    const int b = blockIdx.x, lane = threadIdx.x;
    const int o = lane & 31, tap = b >> 1, i0 = 16 * (b & 1) + 8 * (lane >> 5);
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t lo = f2bf(scale * W[(o * kCnnC + i0 + 2 * q) * kCnnK + tap]);
        const uint32_t hi = f2bf(scale * W[(o * kCnnC + i0 + 2 * q + 1) * kCnnK + tap]);
        w[q] = lo | (hi << 16);
    }
    frag[b * 64 + lane] = make_uint4(w[0], w[1], w[2], w[3]);
}

template <bool SAVE>
__global__ void __launch_bounds__(256) k_conv32_fwd_mfma(const uint16_t* X, const uint4* frag, const float* bias,
                                                         uint16_t* Z, uint16_t* P, int L) {
    __shared__ __attribute__((aligned(16))) uint8_t xs[(kMPos + 8) * kMRow];
    const int g = blockIdx.y;
    const int t0 = blockIdx.x * kMPos;
    const uint16_t* x = X + (int64_t)g * L * kCnnC;
    for (int e = threadIdx.x; e < (kMPos + 8) * 4; e += 256) {
        const int r = e >> 2, q = e & 3;
        const int t = t0 - 4 + r;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (t >= 0 && t < L) v = reinterpret_cast<const uint4*>(x + (int64_t)t * kCnnC)[q];
        *reinterpret_cast<uint4*>(xs + r * kMRow + 16 * q) = v;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint4 a[18];
#pragma unroll
    for (int b = 0; b < 18; ++b) a[b] = frag[b * 64 + lane];
    const int col = lane & 31, hg = lane >> 5;
    float bia[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) bia[e] = bias[8 * (e >> 2) + 4 * hg + (e & 3)];
    __syncthreads();
    for (int tt = 0; tt < 4; ++tt) {
        const int p0 = (w * 4 + tt) * 32;          // tile start inside the workgroup
        if (t0 + p0 >= L) break;
        f32x16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = 0.f;
#pragma unroll
        for (int b = 0; b < 18; ++b) {
            const int tap = b >> 1;
            const uint4 bv = *reinterpret_cast<const uint4*>(xs + (p0 + col + tap) * kMRow + 32 * (b & 1) + 16 * hg);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[b]),
                                                          __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
        }
        // epilogue: lane holds position t = t0 + p0 + col, channels
        // o = 8 (e / 4) + 4 hg + e % 4
        const int t = t0 + p0 + col;
        uint16_t zb[16], pb[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float z = acc[e] + bia[e];
            const float zn = __shfl_xor(z, 1, 64);
            zb[e] = f2bf(z);
            pb[e] = f2bf(0.5f * (fmaxf(z, 0.f) + fmaxf(zn, 0.f)));
        }
        if (t < L) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = 8 * q + 4 * hg;
                if (SAVE)
                    *reinterpret_cast<uint2*>(Z + ((int64_t)g * L + t) * kCnnC + o) =
                        make_uint2((uint32_t)zb[4 * q] | ((uint32_t)zb[4 * q + 1] << 16),
                                   (uint32_t)zb[4 * q + 2] | ((uint32_t)zb[4 * q + 3] << 16));
                if ((t & 1) == 0)
                    *reinterpret_cast<uint2*>(P + ((int64_t)g * (L / 2) + t / 2) * kCnnC + o) =
                        make_uint2((uint32_t)pb[4 * q] | ((uint32_t)pb[4 * q + 1] << 16),
                                   (uint32_t)pb[4 * q + 2] | ((uint32_t)pb[4 * q + 3] << 16));
            }
        }
    }
}

// ------------------------------------------------ inference, all layers --
// Inference in one kernel: a workgroup computes the features of rows u0 ..
// u0 + kFM - 1 of one signal from the input samples they depend on, keeping
// every layer's pooled output in LDS (activations never go to memory).
// Layer l's input rows are taken relative to a_l, with a_4 = u0 and
// a_l = 2 a_{l+1} - 4 (a_0 = 16 u0 - 60): row r of layer l's output (row
// a_{l+1} + r of the next layer's input) pools conv positions cp = 2r and
// 2r + 1, and conv position cp reads input rows cp .. cp + 8. Rows outside
// [0, L_l) are zero at every layer, as in the layer-by-layer kernels.
//
// Layer 0 (one input channel, 9 taps) runs on the matrix cores as a
// contraction 16 deep: the input's Toeplitz matrix (32 positions x 16 taps)
// times W0 (16 taps x 32 channels); tap 9 is the bias (input 1, weight b0),
// taps 10 .. 15 are zero on both sides, so no sample outside a position's
// window enters a product. It rounds differently from the vector-ALU layer 0
// of training, within float32 accumulation. Layers 1 .. 3 run the 18-instruction tiles of
// k_conv32_fwd_mfma in the same order, transposed (see conv_tile), start the
// accumulators at the bias and round to bf16 with the hardware conversion
// (nearest even, as the software rounding for finite values). Weights and
// biases enter halved (exact), so pooling needs no multiplication; halving
// commutes with every rounding here unless a value falls below 2^-126.
//
// Tiles per workgroup (32 conv positions each) and rows kept (each covers
// what the next layer's tiles read):
//   layer 0: 37 tiles -> 592 rows of A1, from 1216 staged samples (< 1200 read)
//   layer 1: 18 tiles -> 288 rows of A2 (296 kept, rows 288 .. 295 zero)
//   layer 2:  9 tiles -> 144 rows of A3 (in A1's space)
//   layer 3:  4 tiles ->  64 feature rows, stored when below F
// The 64 features need A3 rows < 136, A2 rows < 280, A1 rows < 568 and
// samples < 1144, all inside what the tiles compute.
constexpr int kFM = 64;
constexpr int kF0Tiles = 37, kF1Tiles = 18, kF2Tiles = 9, kF3Tiles = 4;
constexpr int kA1Rows = 16 * kF0Tiles, kA2Rows = 296, kX0N = 1216;
constexpr int kFusedLds = 2 * kX0N * 2 + (kA1Rows + kA2Rows) * kMRow + 4 * kCnnC * 4;
static_assert(16 * kF2Tiles <= kA1Rows, "A3 fits in A1's space");
static_assert(32 * kF1Tiles + 8 <= kA1Rows && 32 * kF2Tiles + 8 <= kA2Rows && 32 * kF3Tiles + 8 <= 16 * kF2Tiles,
              "each layer's tiles read kept rows");
static_assert(32 * kF0Tiles + 16 <= kX0N, "layer 0 reads staged samples");
// A1 rows from which layer 2's weight fragments (18 KB) are kept: past the
// rows layer 2 writes (A3), inside A1; A2 holds layer 1's and layer 3's,
// clear of its zeroed tail rows
constexpr int kFragRowA1 = 152;
static_assert(16 * kF2Tiles + 8 <= kFragRowA1 && kFragRowA1 * kMRow + 18 * 64 * 16 <= kA1Rows * kMRow,
              "layer 2's fragments sit in A1 past A3");
static_assert(18 * 64 * 16 <= 16 * kF1Tiles * kMRow, "layer 1's and 3's fragments sit in A2 before its zeroed rows");
static_assert((2 * kX0N * 2) % 16 == 0 && (kFragRowA1 * kMRow) % 16 == 0 && (kA1Rows * kMRow) % 16 == 0,
              "fragment areas are 16-byte aligned");

__device__ __forceinline__ float dpp_xor1(float v) {
    // quad_perm [1,0,3,2]: lane l ^ 1 (every lane has a source, so bound_ctrl
    // changes nothing; it lets the move fold into the addition)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xf, 0xf, true));
}

// The fused kernel computes each tile transposed: C[t][o] = sum_k X[t][k]
// W[k][o] with the input fragment as the first operand and the weights as
// the second (the two operands of v_mfma_f32_32x32x16_bf16 have the same
// lane layout, so the fragments are those of k_conv32_fwd_mfma). Lane l then
// holds channel o = l % 32 of conv positions p0 + 8 (e / 4) + 4 (l / 32) +
// e % 4: the two positions of a pooled row sit in one lane (e, e + 1 for
// even e), and the lane's bias is one value.
//
// One layer-1..3 tile: conv positions p0 .. p0 + 31 from input rows in LDS,
// accumulated onto the bias (acc holds the lane's bias on entry).
__device__ __forceinline__ f32x16 conv_tile(const uint8_t* in, const uint4 (&a)[18], int p0, int col, int hg,
                                            f32x16 acc) {
#pragma unroll
    for (int b = 0; b < 18; ++b) {
        const int tap = b >> 1;
        const uint4 bv = *reinterpret_cast<const uint4*>(in + (p0 + col + tap) * kMRow + 32 * (b & 1) + 16 * hg);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, bv), __builtin_bit_cast(bf16x8, a[b]),
                                                      acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ f32x16 splat16(float v) {
    f32x16 acc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = v;
    return acc;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// ReLU as an integer maximum of the bit pattern with 0: every negative value
// (-0 included) becomes +0, every other value stays.
__device__ __forceinline__ float relu_bits(float v) {
    return __builtin_bit_cast(float, max(__builtin_bit_cast(int, v), 0));
}

// ReLU and pooling of a transposed tile. The accumulators hold z / 2
// (weights and bias halved, exact), so relu(z/2) + relu(z'/2) = (relu(z) +
// relu(z')) / 2, the pooled value. Dword q holds pooled rows
// p0 / 2 + 4 q + 2 hg and the next one (low and high bf16, rounded to
// nearest even) of the lane's channel.
__device__ __forceinline__ void tile_pool(const f32x16& acc, uint32_t (&pk)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float r0 = relu_bits(acc[4 * q]) + relu_bits(acc[4 * q + 1]);
        const float r1 = relu_bits(acc[4 * q + 2]) + relu_bits(acc[4 * q + 3]);
        const f32x2_t p = {r0, r1};
        pk[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(p, bf16x2_t));
    }
}

// Pooled rows into LDS: zeros where a row's absolute index a_out + row is
// outside [0, Lout) (only tiles at the signal's ends have such rows).
__device__ __forceinline__ void pool_to_lds(const f32x16& acc, int p0, int col, int hg, uint8_t* out, int a_out,
                                            int Lout) {
    uint32_t pk[4];
    tile_pool(acc, pk);
    const int r0 = p0 / 2 + 2 * hg;
    uint8_t* dst = out + r0 * kMRow + 2 * col;
    const int first = a_out + p0 / 2;
    if (first >= 0 && first + 16 <= Lout) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<uint16_t*>(dst + 4 * q * kMRow) = (uint16_t)pk[q];
            *reinterpret_cast<uint16_t*>(dst + (4 * q + 1) * kMRow) = (uint16_t)(pk[q] >> 16);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ab = a_out + r0 + 4 * q;
            const bool ok0 = ab >= 0 && ab < Lout, ok1 = ab + 1 >= 0 && ab + 1 < Lout;
            *reinterpret_cast<uint16_t*>(dst + 4 * q * kMRow) = ok0 ? (uint16_t)pk[q] : (uint16_t)0;
            *reinterpret_cast<uint16_t*>(dst + (4 * q + 1) * kMRow) = ok1 ? (uint16_t)(pk[q] >> 16) : (uint16_t)0;
        }
    }
}

constexpr int kFusedWaves = 8;     // waves per workgroup (two workgroups per CU by LDS)

__global__ void __launch_bounds__(64 * kFusedWaves) k_cnn_fwd_fused(
    const uint16_t* __restrict__ X0, const float* __restrict__ W0, const float* __restrict__ b0,
    const uint4* __restrict__ frag, const float* __restrict__ bias1, const float* __restrict__ bias2,
    const float* __restrict__ bias3, uint16_t* __restrict__ Fout, int L0) {
    constexpr int NT = 64 * kFusedWaves;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    uint16_t* x0e = reinterpret_cast<uint16_t*>(lds);     // x0e[i] = input sample a_0 + i
    uint16_t* x0o = x0e + kX0N;                            // x0o[i] = input sample a_0 + i + 1
    uint8_t* a1 = lds + 2 * kX0N * 2;
    uint8_t* a2 = a1 + kA1Rows * kMRow;
    uint8_t* a3 = a1;                                      // layer 2 writes after layer 1 has read A1
    float* sb = reinterpret_cast<float*>(a2 + kA2Rows * kMRow);   // biases, [layer][32]
    const int g = blockIdx.y, u0 = blockIdx.x * kFM;
    const int L1 = L0 / 2, L2 = L0 / 4, L3 = L0 / 8, F = L0 / 16;
    const int s0 = 16 * u0 - 60, s1 = 8 * u0 - 28, s2 = 4 * u0 - 12, s3 = 2 * u0 - 4;
    const uint16_t* x = X0 + (int64_t)g * L0;
    const int tid = threadIdx.x;
    for (int i = tid; i <= kX0N; i += NT) {
        const int t = s0 + i;
        const uint16_t v = (t >= 0 && t < L0) ? x[t] : (uint16_t)0;
        if (i < kX0N) x0e[i] = v;
        if (i > 0) x0o[i - 1] = v;
    }
    if (tid < 4 * kCnnC) {
        const int l = tid / kCnnC, o = tid % kCnnC;
        sb[tid] = 0.5f * (l == 0 ? b0 : l == 1 ? bias1 : l == 2 ? bias2 : bias3)[o];
    }
    for (int e = tid; e < (kA2Rows - 16 * kF1Tiles) * 4; e += NT)
        *reinterpret_cast<uint4*>(a2 + (16 * kF1Tiles + (e >> 2)) * kMRow + 16 * (e & 3)) = make_uint4(0, 0, 0, 0);
    const int lane = tid & 63, w = tid >> 6, col = lane & 31, hg = lane >> 5;
    // layer 0's weight fragment: channel col, taps 8 hg .. 8 hg + 7; tap 9
    // carries the bias (its input is 1), taps 10 .. 15 are zero
    uint32_t w0p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k0 = 8 * hg + 2 * q, k1 = k0 + 1;
        auto wk = [&](int k) -> uint32_t {
            return k < kCnnK ? f2bf(0.5f * W0[col * kCnnK + k]) : k == kCnnK ? f2bf(0.5f * b0[col]) : 0u;
        };
        w0p[q] = wk(k0) | (wk(k1) << 16);
    }
    const uint4 a0f = make_uint4(w0p[0], w0p[1], w0p[2], w0p[3]);
    // A layer's 18 weight fragments (18 KB) are copied once per workgroup
    // into LDS the layer does not touch, and every wave takes its registers'
    // copy from there: loaded by each wave from memory they cost the
    // vector-memory data path eight times their size. Layer 1's go into A2
    // (written only by layer 1), layer 2's into A1 past the rows of A3,
    // layer 3's into A2 again.
    uint4 wf[18];
    frag += (size_t)(kCnnLayers - 1) * 18 * 64;               // the halved fragments
    uint4* fl_a2 = reinterpret_cast<uint4*>(a2);
    uint4* fl_a1 = reinterpret_cast<uint4*>(a1 + kFragRowA1 * kMRow);
    auto stage_frags = [&](const uint4* src, uint4* dst) {
        for (int e = tid; e < 18 * 64; e += NT) dst[e] = src[e];
    };
    auto take_frags = [&](const uint4* src) {
#pragma unroll
        for (int b = 0; b < 18; ++b) wf[b] = src[b * 64 + lane];
    };
    stage_frags(frag, fl_a2);
    __syncthreads();
    // layer 0 -> A1
    for (int t = w; t < kF0Tiles; t += kFusedWaves) {
        const int p0 = 32 * t, base = p0 + col + 8 * hg;
        const uint32_t* src = reinterpret_cast<const uint32_t*>((base & 1) ? x0o + (base - 1) : x0e + base);
        uint4 bv = make_uint4(src[0], src[1], src[2], src[3]);
        if (hg) bv = make_uint4((bv.x & 0xffffu) | 0x3f800000u, 0u, 0u, 0u);   // tap 8, then 1.0 for the bias
        const f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, bv), __builtin_bit_cast(bf16x8, a0f), splat16(0.f), 0, 0, 0);
        pool_to_lds(acc, p0, col, hg, a1, s1, L1);
    }
    take_frags(fl_a2);
    lds_barrier();                                  // A1 complete, layer 1's fragments taken from A2
    // layer 1 -> A2
    for (int t = w; t < kF1Tiles; t += kFusedWaves)
        pool_to_lds(conv_tile(a1, wf, 32 * t, col, hg, splat16(sb[kCnnC + col])), 32 * t, col, hg, a2, s2, L2);
    lds_barrier();                                  // A1 read, A2 complete
    stage_frags(frag + 18 * 64, fl_a1);
    lds_barrier();
    take_frags(fl_a1);
    // layer 2 -> A3 (A1's first rows, below layer 2's fragments)
    for (int t = w; t < kF2Tiles; t += kFusedWaves)
        pool_to_lds(conv_tile(a2, wf, 32 * t, col, hg, splat16(sb[2 * kCnnC + col])), 32 * t, col, hg, a3, s3,
                    L3);
    lds_barrier();                                  // A2 read, A3 complete
    stage_frags(frag + 36 * 64, fl_a2);
    lds_barrier();
    if (w < kF3Tiles) take_frags(fl_a2);            // waves without a layer-3 tile need none
    // layer 3 -> features
    for (int t = w; t < kF3Tiles; t += kFusedWaves) {
        const int p0 = 32 * t;
        uint32_t pk[4];
        tile_pool(conv_tile(a3, wf, p0, col, hg, splat16(sb[3 * kCnnC + col])), pk);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = p0 / 2 + 2 * hg + 4 * q + h;
                if (u0 + row < F)
                    Fout[((int64_t)g * F + u0 + row) * kCnnC + col] = (uint16_t)(h ? pk[q] >> 16 : pk[q]);
            }
    }
}

// ----------------------------------------------------------------- head --
constexpr int kHeadWaves = 8;     // waves per workgroup (one workgroup per pair)
// raw[b][k] = sum_t sum_c Fx[t][c] Fy[t + s][c], s = k - nb/2, on the bf16
// matrix cores. For a fixed block offset D, the 32 x 32 products
// C_I[i][j] = <Fx[32 I + i], Fy[32 (I + D) + j]> all belong to the shifts
// s = j - i + 32 D, so one accumulator per D sums them over every row block
// I (two instructions of 16 channels each). The diagonals of the D tiles are
// then added in a fixed order (deterministic). One workgroup per pair.
__global__ void __launch_bounds__(64 * kHeadWaves) k_head_fwd(const uint16_t* __restrict__ Fe, const float* params_alpha, float* raw,
                                                  float* logits, int F, int nb) {
    extern __shared__ float tiles[];                 // [nD][32][32]
    const int b = blockIdx.x;
    const int h = nb / 2;
    const int dmin = -(h / 32), nD = nb / 32 + 1;
    const int nblk = F / 32;
    const uint8_t* fx = reinterpret_cast<const uint8_t*>(Fe + (int64_t)(2 * b) * F * kCnnC);
    const uint8_t* fy = reinterpret_cast<const uint8_t*>(Fe + (int64_t)(2 * b + 1) * F * kCnnC);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31, g = lane >> 5;
    // wave w takes a contiguous range of offsets, kHD at a time: the Fx row
    // block I is loaded once for all of them, and the Fy blocks I + D of
    // neighbouring offsets are neighbours (cache hits). Each accumulator
    // still sums I in increasing order, two instructions per block.
    constexpr int kHD = 3;
    const int per = (nD + kHeadWaves - 1) / kHeadWaves;
    const int d_end = min(nD, (w + 1) * per);
    for (int c0 = w * per; c0 < d_end; c0 += kHD) {
        const int cnt = min(kHD, d_end - c0), D0 = dmin + c0;
        f32x16 acc[kHD];
#pragma unroll
        for (int k = 0; k < kHD; ++k)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[k][e] = 0.f;
        const int ilo = max(0, -(D0 + cnt - 1)), ihi = min(nblk, nblk - D0);
        for (int I = ilo; I < ihi; ++I) {
            uint4 av[2], bv[kHD][2];
            const uint8_t* ax = fx + (int64_t)(32 * I + r) * 64 + 16 * g;
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) av[kb] = *reinterpret_cast<const uint4*>(ax + 32 * kb);
#pragma unroll
            for (int k = 0; k < kHD; ++k) {
                const int J = I + D0 + k;
                if (k < cnt && J >= 0 && J < nblk) {
                    const uint8_t* by = fy + (int64_t)(32 * J + r) * 64 + 16 * g;
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb) bv[k][kb] = *reinterpret_cast<const uint4*>(by + 32 * kb);
                }
            }
#pragma unroll
            for (int k = 0; k < kHD; ++k) {
                const int J = I + D0 + k;
                if (k < cnt && J >= 0 && J < nblk) {
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb)
                        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[kb]),
                                                                         __builtin_bit_cast(bf16x8, bv[k][kb]), acc[k],
                                                                         0, 0, 0);
                }
            }
        }
        // lane holds column j = r, rows i = 8 (e / 4) + 4 g + e % 4
#pragma unroll
        for (int k = 0; k < kHD; ++k)
            if (k < cnt) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    tiles[((c0 + k) * 32 + 8 * (e >> 2) + 4 * g + (e & 3)) * 32 + r] = acc[k][e];
            }
    }
    __syncthreads();
    const float a = *params_alpha;
    for (int k = threadIdx.x; k < nb; k += 64 * kHeadWaves) {
        const int sft = k - h;
        float sum = 0.f;
        for (int di = 0; di < nD; ++di) {
            const int dlt = sft - 32 * (dmin + di);        // j - i
            if (dlt < -31 || dlt > 31) continue;
            const int i0 = dlt < 0 ? -dlt : 0, i1 = dlt < 0 ? 32 : 32 - dlt;
            for (int i = i0; i < i1; ++i) sum += tiles[(di * 32 + i) * 32 + i + dlt];
        }
        raw[(int64_t)b * nb + k] = sum;
        logits[(int64_t)b * nb + k] = a * sum;
    }
}

// ------------------------------------------------ softmax, loss, top-k --
// One workgroup per pair. Training (labels set): loss, dlog = (softmax -
// onehot) / B and dalpha_b = sum dlog raw. Proposal (top set): the top-k
// bins (ties to the smaller bin) and margin = logit_(1) - logit_(k+1).
__global__ void __launch_bounds__(256) k_softmax_topk(const float* logits, const float* raw, const int32_t* labels,
                                                      int nb, float inv_b, float* loss, float* dlog, float* dalpha,
                                                      int topk, int32_t* top, float* margin) {
    const int b = blockIdx.x;
    const float* z = logits + (int64_t)b * nb;
    __shared__ float sv[256];
    __shared__ int si[256];
    __shared__ float s_max, s_sum;
    const int t = threadIdx.x;
    // max
    float m = -INFINITY;
    for (int k = t; k < nb; k += 256) m = fmaxf(m, z[k]);
    sv[t] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) sv[t] = fmaxf(sv[t], sv[t + o]);
        __syncthreads();
    }
    if (t == 0) s_max = sv[0];
    __syncthreads();
    const float mx = s_max;
    if (labels) {
        float s = 0.f;
        for (int k = t; k < nb; k += 256) s += __expf(z[k] - mx);
        __syncthreads();
        sv[t] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) sv[t] += sv[t + o];
            __syncthreads();
        }
        if (t == 0) s_sum = sv[0];
        __syncthreads();
        const float S = s_sum;
        const int lab = labels[b];
        float da = 0.f;
        for (int k = t; k < nb; k += 256) {
            const float pr = __expf(z[k] - mx) / S;
            const float g = (pr - (k == lab ? 1.f : 0.f)) * inv_b;
            dlog[(int64_t)b * nb + k] = g;
            da += g * raw[(int64_t)b * nb + k];
        }
        __syncthreads();
        sv[t] = da;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) sv[t] += sv[t + o];
            __syncthreads();
        }
        if (t == 0) {
            dalpha[b] = sv[0];
            loss[b] = -(z[lab] - mx - __logf(S));
        }
    }
    if (top) {
        // k+1 rounds of (max, smallest index) over the bins not yet taken
        __shared__ int taken[kCnnMaxTop + 1];
        float first = 0.f;
        for (int r = 0; r <= topk; ++r) {
            float bv = -INFINITY;
            int bi = INT32_MAX;
            for (int k = t; k < nb; k += 256) {
                bool used = false;
                for (int j = 0; j < r; ++j) used |= taken[j] == k;
                if (used) continue;
                const float v = z[k];
                if (v > bv || (v == bv && k < bi)) {
                    bv = v;
                    bi = k;
                }
            }
            __syncthreads();
            sv[t] = bv;
            si[t] = bi;
            __syncthreads();
            for (int o = 128; o > 0; o >>= 1) {
                if (t < o) {
                    const float v2 = sv[t + o];
                    const int i2 = si[t + o];
                    if (v2 > sv[t] || (v2 == sv[t] && i2 < si[t])) {
                        sv[t] = v2;
                        si[t] = i2;
                    }
                }
                __syncthreads();
            }
            if (t == 0) taken[r] = si[0];
            if (r == 0) first = sv[0];
            if (r == topk && t == 0) margin[b] = si[0] == INT32_MAX ? INFINITY : first - sv[0];
            __syncthreads();
        }
        if (t < topk) top[(int64_t)b * topk + t] = taken[t];
    }
}

// Proposal only: one wave per pair holds the pair's logits in registers
// (bin lane + 64 j in v[j]) and takes k + 1 rounds of (max, smallest bin)
// over the bins not yet taken, by shuffles; the same choices and margin as
// the proposal path of k_softmax_topk.
constexpr int kTopPerLane = 16;             // bins per lane: nb <= 1024
__global__ void __launch_bounds__(256) k_topk_wave(const float* __restrict__ logits, int B, int nb, int topk,
                                                   int32_t* __restrict__ top, float* __restrict__ margin) {
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;                     // the whole wave
    const float* z = logits + (int64_t)b * nb;
    float v[kTopPerLane];
#pragma unroll
    for (int j = 0; j < kTopPerLane; ++j) {
        const int k = lane + 64 * j;
        v[j] = k < nb ? z[k] : 0.f;
    }
    uint32_t taken = 0;                     // bit j: bin lane + 64 j is taken
    float first = 0.f;
    for (int r = 0; r <= topk; ++r) {
        float bv = -INFINITY;
        int bi = INT32_MAX;
#pragma unroll
        for (int j = 0; j < kTopPerLane; ++j) {
            const int k = lane + 64 * j;
            if (k < nb && !((taken >> j) & 1u) && (v[j] > bv || (v[j] == bv && k < bi))) {
                bv = v[j];
                bi = k;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const float v2 = __shfl_xor(bv, o, 64);
            const int i2 = __shfl_xor(bi, o, 64);
            if (v2 > bv || (v2 == bv && i2 < bi)) {
                bv = v2;
                bi = i2;
            }
        }
        if (bi != INT32_MAX && (bi & 63) == lane) taken |= 1u << (bi >> 6);
        if (r == 0) first = bv;
        if (lane == 0) {
            if (r < topk) top[(int64_t)b * topk + r] = bi;
            else margin[b] = bi == INT32_MAX ? INFINITY : first - bv;
        }
    }
}

// ------------------------------------------------------------ head bwd --
// dFx[t][c] = alpha sum_k dlog[k] Fy[t + k - h][c]
// dFy[t][c] = alpha sum_k dlog[k] Fx[t - k + h][c]
// grid (F / 64, B, 2 sides); thread -> position (0..63) and 8 channels.
__global__ void __launch_bounds__(256) k_head_bwd(const uint16_t* Fe, const float* dlog, const float* params_alpha,
                                                  float* dFe, int F, int nb) {
    extern __shared__ float hb[];
    const int b = blockIdx.y, side = blockIdx.z;
    const int t0 = blockIdx.x * 64;
    const int h = nb / 2;
    float* sd = hb;                                  // dlog [nb]
    uint16_t* so = reinterpret_cast<uint16_t*>(hb + nb);   // other side's window
    const uint16_t* other = Fe + (int64_t)(2 * b + (1 - side)) * F * kCnnC;
    // side 0 needs Fy rows t + k - h, k in [0, nb): rows [t0 - h, t0 + 63 - h + nb - 1]
    // side 1 needs Fx rows t - k + h: rows [t0 + h - nb + 1, t0 + 63 + h]
    const int wlo = side == 0 ? t0 - h : t0 + h - nb + 1;
    const int nw = 64 + nb - 1;
    for (int k = threadIdx.x; k < nb; k += 256) sd[k] = dlog[(int64_t)b * nb + k];
    for (int e = threadIdx.x; e < nw * 4; e += 256) {
        const int r = e >> 2, q = e & 3;
        const int t = wlo + r;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (t >= 0 && t < F) v = reinterpret_cast<const uint4*>(other + (int64_t)t * kCnnC)[q];
        reinterpret_cast<uint4*>(so)[e] = v;
    }
    __syncthreads();
    const int tp = threadIdx.x & 63, cg = threadIdx.x >> 6;
    const int t = t0 + tp;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < nb; ++k) {
        // window row of the partner position
        const int r = side == 0 ? (t + k - h) - wlo : (t - k + h) - wlo;
        const uint4 v = reinterpret_cast<const uint4*>(so + r * kCnnC)[cg];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        const float d = sd[k];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            acc[2 * e] += d * __uint_as_float(w[e] << 16);
            acc[2 * e + 1] += d * __uint_as_float(w[e] & 0xFFFF0000u);
        }
    }
    if (t >= F) return;
    const float a = *params_alpha;
    float* dst = dFe + ((int64_t)(2 * b + side) * F + t) * kCnnC + cg * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) dst[c] = a * acc[c];
}

// ------------------------------------------------- conv backward (data) --
// dZ[t][o] = dP[t/2][o] / 2 * (Z[t][o] > 0); dX[t][i] = sum_o sum_k
// W[o][i][k] dZ[t + 4 - k][o]. grid (L / 128, nsig), thread -> 2 positions
// and 8 input channels.
__global__ void __launch_bounds__(256) k_conv32_bwd_data(const float* dP, const uint16_t* Z, const float* W,
                                                         float* dX, int L) {
    __shared__ float dz[kCnnC][kXs + 1];
    __shared__ float ws[kCnnK][kCnnC][kCnnC];   // [k][co][ci]
    const int g = blockIdx.y;
    const int t0 = blockIdx.x * kTile;
    for (int e = threadIdx.x; e < kXs * kCnnC; e += 256) {
        const int r = e / kCnnC, c = e % kCnnC;
        const int t = t0 - 4 + r;
        float v = 0.f;
        if (t >= 0 && t < L) {
            const float z = bf2f(Z[((int64_t)g * L + t) * kCnnC + c]);
            if (z > 0.f) v = 0.5f * dP[((int64_t)g * (L / 2) + t / 2) * kCnnC + c];
        }
        dz[c][r] = v;
    }
    for (int e = threadIdx.x; e < kCnnC * kCnnC * kCnnK; e += 256) {
        const int co = e / (kCnnC * kCnnK), rem = e % (kCnnC * kCnnK);
        const int ci = rem / kCnnK, k = rem % kCnnK;
        ws[k][co][ci] = W[e];
    }
    __syncthreads();
    const int tp = threadIdx.x & 63, cg = threadIdx.x >> 6;
    float acc[2][8] = {};
    for (int co = 0; co < kCnnC; ++co) {
        float zv[10];
        // dZ rows t + 4 - k for t = 2tp, 2tp+1 (tile coordinates: + 4)
#pragma unroll
        for (int j = 0; j < 10; ++j) zv[j] = dz[co][2 * tp + j];
#pragma unroll
        for (int k = 0; k < kCnnK; ++k) {
            const float4 wa = *reinterpret_cast<const float4*>(&ws[k][co][cg * 8]);
            const float4 wb = *reinterpret_cast<const float4*>(&ws[k][co][cg * 8 + 4]);
            const float w8[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
            // tile row of dZ[t + 4 - k] is (t - t0) + 8 - k
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                acc[0][c] += w8[c] * zv[8 - k];
                acc[1][c] += w8[c] * zv[9 - k];
            }
        }
    }
    const int tc = t0 + 2 * tp;
    if (tc >= L) return;
    float* d0 = dX + ((int64_t)g * L + tc) * kCnnC + cg * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        d0[c] = acc[0][c];
        d0[kCnnC + c] = acc[1][c];
    }
}

// ----------------------------------------------- conv backward (weights) --
// Per workgroup (signal g, chunk of kWChunk positions): partial dW[o][i][k]
// = sum_t dZ[t][o] X[t + k - 4][i] and db[o] = sum_t dZ[t][o], written to
// part[blk][n] with n = 32 cin 9 + 32. Thread -> o = t % 32 and a group of
// cin/8 input channels (cin = 32) or one (o, k) slot pair (cin = 1).
constexpr int kWChunk = 512;

template <int CIN>
__global__ void __launch_bounds__(256) k_conv_bwd_w(const float* dP, const uint16_t* Z, const uint16_t* X, int L,
                                                    float* part) {
    constexpr int NW = kCnnC * CIN * kCnnK;
    __shared__ float dz[64][kCnnC + 1];
    __shared__ float xs[64 + 8][CIN == 1 ? 1 : kCnnC + 1];
    const int g = blockIdx.y;
    const int nchunk = gridDim.x;
    const int c0 = blockIdx.x * kWChunk;
    const int o = threadIdx.x & 31;
    const int grp = threadIdx.x >> 5;          // 0..7
    constexpr int NI = CIN == 1 ? 1 : CIN / 8;
    float acc[NI][kCnnK] = {};
    float accb = 0.f;
    // cin = 1: thread (o, grp) owns tap k = grp (and grp 0 also tap 8)
    float acc8 = 0.f;
    for (int tb = c0; tb < c0 + kWChunk && tb < L; tb += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * kCnnC; e += 256) {
            const int r = e / kCnnC, c = e % kCnnC;
            const int t = tb + r;
            float v = 0.f;
            if (t < L) {
                const float z = bf2f(Z[((int64_t)g * L + t) * kCnnC + c]);
                if (z > 0.f) v = 0.5f * dP[((int64_t)g * (L / 2) + t / 2) * kCnnC + c];
            }
            dz[r][c] = v;
        }
        for (int e = threadIdx.x; e < 72 * CIN; e += 256) {
            const int r = e / CIN, c = e % CIN;
            const int t = tb - 4 + r;
            float v = 0.f;
            if (t >= 0 && t < L) v = bf2f(X[((int64_t)g * L + t) * CIN + c]);
            xs[r][CIN == 1 ? 0 : c] = v;
        }
        __syncthreads();
        for (int r = 0; r < 64; ++r) {
            const float d = dz[r][o];
            if (CIN == 1) {
                acc[0][0] += d * xs[r + grp][0];
                if (grp == 0) acc8 += d * xs[r + 8][0];
            } else {
#pragma unroll
                for (int ii = 0; ii < NI; ++ii) {
#pragma unroll
                    for (int k = 0; k < kCnnK; ++k) acc[ii][k] += d * xs[r + k][grp * NI + ii];
                }
            }
            if (grp == 0) accb += d;
        }
    }
    float* dst = part + ((int64_t)g * nchunk + blockIdx.x) * (NW + kCnnC);
    if (CIN == 1) {
        dst[o * kCnnK + grp] = acc[0][0];
        if (grp == 0) dst[o * kCnnK + 8] = acc8;
    } else {
#pragma unroll
        for (int ii = 0; ii < NI; ++ii)
#pragma unroll
            for (int k = 0; k < kCnnK; ++k) dst[(o * CIN + grp * NI + ii) * kCnnK + k] = acc[ii][k];
    }
    if (grp == 0) dst[NW + o] = accb;
}

// grad[i] = sum_b part[b][i] (fixed order); one thread per element.
__global__ void k_reduce_parts(const float* part, int nblk, int n, float* grad) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * n + i];
    grad[i] = s;
}

// --------------------------------------------------------------- Adam --
// Updates the fp32 masters and refreshes their bf16-rounded copies.
__global__ void k_adam(float* p, const float* g, float* m, float* v, float* wc, int n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    wc[i] = i == n - 1 ? pi : bf16_round_dev(pi);     // alpha (last) stays float32
}

__global__ void k_round_copy(const float* p, float* wc, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) wc[i] = i == n - 1 ? p[i] : bf16_round_dev(p[i]);
}

// ---------------------------------------------------------------- host --

int cnn_param_count(int layers) { return kCnnC * 1 * kCnnK + kCnnC + (layers - 1) * (kCnnC * kCnnC * kCnnK + kCnnC) + 1; }

size_t cnn_param_offset(int layer) {
    if (layer == 0) return 0;
    return (size_t)(kCnnC * kCnnK + kCnnC) + (size_t)(layer - 1) * (kCnnC * kCnnC * kCnnK + kCnnC);
}

int launch_cnn_decimate(const CnnSig* sigs, int nsig, int ld, uint16_t* out, hipStream_t s) {
    if (nsig == 0) return TDE_OK;
    hipLaunchKernelGGL(k_cnn_decimate, dim3(ceil_div(ld, 256), nsig), dim3(256), 0, s, sigs, ld, out);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

// Forward through the encoder and head for nsig = 2 B signals. acts: Z_l
// (may be null: inference) and X_l per layer; logits and raw [B][nb].
int launch_cnn_forward(const CnnNet& net, const float* wc, const uint16_t* xdec, int B, CnnActs& A, float* raw,
                       float* logits, hipStream_t s) {
    const int nsig = 2 * B;
    int L = net.ld;
    const uint16_t* X = xdec;
    for (int l = 0; l < kCnnLayers; ++l) {
        const float* W = wc + cnn_param_offset(l);
        const float* bias = W + (l == 0 ? kCnnC * kCnnK : kCnnC * kCnnC * kCnnK);
        uint16_t* Z = A.z[l];
        uint16_t* P = A.x[l + 1];
        if (l == 0 && kCnnLayers == 4 && !A.z[0] && !A.z[1] && !A.z[2] && !A.z[3]) {
            // inference: all four layers in one pass (activations stay in LDS)
            static bool lds_attr = false;
            if (!lds_attr) {
                TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_cnn_fwd_fused,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, kFusedLds));
                lds_attr = true;
            }
            const float* bl[4];
            for (int k = 1; k < 4; ++k) bl[k] = wc + cnn_param_offset(k) + kCnnC * kCnnC * kCnnK;
            const uint4* fr = reinterpret_cast<const uint4*>(net.frag);
            hipLaunchKernelGGL(k_cnn_fwd_fused, dim3(ceil_div(L / 16, kFM), nsig), dim3(64 * kFusedWaves), kFusedLds, s,
                               X, W, bias,
                               fr, bl[1], bl[2], bl[3], A.x[4], L);
            TDE_HIP_CHECK(hipGetLastError());
            X = A.x[4];
            L /= 16;
            break;
        }
        if (l == 0) {
            if (Z) hipLaunchKernelGGL(k_conv1_fwd<true>, dim3(ceil_div(L / 2, 256), nsig), dim3(256), 0, s, X, W, bias, Z, P, L);
            else hipLaunchKernelGGL(k_conv1_fwd<false>, dim3(ceil_div(L / 2, 256), nsig), dim3(256), 0, s, X, W, bias, Z, P, L);
        } else {
            const uint4* fr = reinterpret_cast<const uint4*>(net.frag) + (size_t)(l - 1) * 18 * 64;
            if (Z)
                hipLaunchKernelGGL(k_conv32_fwd_mfma<true>, dim3(ceil_div(L, kMPos), nsig), dim3(256), 0, s, X, fr,
                                   bias, Z, P, L);
            else
                hipLaunchKernelGGL(k_conv32_fwd_mfma<false>, dim3(ceil_div(L, kMPos), nsig), dim3(256), 0, s, X, fr,
                                   bias, Z, P, L);
        }
        TDE_HIP_CHECK(hipGetLastError());
        X = P;
        L /= 2;
    }
    const int F = L;
    const size_t hl = (size_t)(net.nb / 32 + 1) * 32 * 32 * 4;
    static bool attr = false;
    if (!attr) {
        TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_head_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        TDE_HIP_CHECK(hipFuncSetAttribute((const void*)k_head_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
        attr = true;
    }
    hipLaunchKernelGGL(k_head_fwd, dim3(B), dim3(64 * kHeadWaves), hl, s, X, wc + net.nparams - 1, raw, logits, F, net.nb);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_cnn_topk(const float* logits, int B, int nb, int topk, int32_t* top, float* margin, hipStream_t s) {
    if (nb > 64 * kTopPerLane) return set_error(TDE_ERR_ARG, "cnn top-k: more than %d bins", 64 * kTopPerLane);
    hipLaunchKernelGGL(k_topk_wave, dim3(ceil_div(B, 4)), dim3(256), 0, s, logits, B, nb, topk, top, margin);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

// Loss, gradients (into grad, the flat parameter layout) of the mean loss.
int launch_cnn_backward(const CnnNet& net, const float* wc, int B, const int32_t* labels, CnnActs& A,
                        const float* raw, const float* logits, CnnGrad& G, hipStream_t s) {
    const int nsig = 2 * B;
    const int F = net.ld >> kCnnLayers;
    hipLaunchKernelGGL(k_softmax_topk, dim3(B), dim3(256), 0, s, logits, raw, labels, net.nb, 1.f / B, G.loss,
                       G.dlog, G.dalpha, 0, nullptr, nullptr);
    TDE_HIP_CHECK(hipGetLastError());
    const size_t hl = (size_t)net.nb * 4 + (size_t)(64 + net.nb) * kCnnC * 2;
    hipLaunchKernelGGL(k_head_bwd, dim3(ceil_div(F, 64), B, 2), dim3(256), hl, s, A.x[kCnnLayers], G.dlog,
                       wc + net.nparams - 1, G.dx[kCnnLayers], F, net.nb);
    TDE_HIP_CHECK(hipGetLastError());
    for (int l = kCnnLayers - 1; l >= 0; --l) {
        const int L = net.ld >> l;
        const float* W = wc + cnn_param_offset(l);
        const float* dP = G.dx[l + 1];
        const int nchunk = (int)ceil_div(L, kWChunk);
        const int cin = l == 0 ? 1 : kCnnC;
        const int n = kCnnC * cin * kCnnK + kCnnC;
        if (l == 0)
            hipLaunchKernelGGL(k_conv_bwd_w<1>, dim3(nchunk, nsig), dim3(256), 0, s, dP, A.z[l], A.x[l], L, G.part);
        else
            hipLaunchKernelGGL(k_conv_bwd_w<kCnnC>, dim3(nchunk, nsig), dim3(256), 0, s, dP, A.z[l], A.x[l], L, G.part);
        TDE_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_reduce_parts, dim3(ceil_div(n, 256)), dim3(256), 0, s, G.part, nchunk * nsig, n,
                           G.grad + cnn_param_offset(l));
        TDE_HIP_CHECK(hipGetLastError());
        if (l > 0) {
            hipLaunchKernelGGL(k_conv32_bwd_data, dim3(ceil_div(L, kTile), nsig), dim3(256), 0, s, dP, A.z[l], W,
                               G.dx[l], L);
            TDE_HIP_CHECK(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, s, G.dalpha, B, 1, G.grad + net.nparams - 1);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_adam(float* p, const float* g, float* m, float* v, float* wc, int n, float lr, int step,
                hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, g, m, v, wc, n, lr, b1, b2, 1e-8f, bc1,
                       bc2);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

int launch_round_copy(const float* p, float* wc, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_round_copy, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, wc, n);
    TDE_HIP_CHECK(hipGetLastError());
    return TDE_OK;
}

// Per-lane matrix-core fragments of the 32 -> 32 layers' bf16 weights.
// The second half holds the same fragments of W / 2 (the fused inference
// kernel's, see there).
int launch_pack_frags(const float* wc, void* frag, hipStream_t s) {
    for (int h = 0; h < 2; ++h)
        for (int l = 1; l < kCnnLayers; ++l) {
            hipLaunchKernelGGL(k_pack_wfrag, dim3(18), dim3(64), 0, s, wc + cnn_param_offset(l),
                               reinterpret_cast<uint4*>(frag) + (size_t)(h * (kCnnLayers - 1) + l - 1) * 18 * 64,
                               h ? 0.5f : 1.f);
            TDE_HIP_CHECK(hipGetLastError());
        }
    return TDE_OK;
}

}  // namespace tde
