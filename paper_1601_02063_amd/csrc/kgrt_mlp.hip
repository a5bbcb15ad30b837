// kgrt_mlp.hip -- the learned surrogate: a 4-256-256-256-256-5 SiLU perceptron
// trained and evaluated by hand-written kernels on v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation; the 4-wide input layer and the 5-wide
// output head also run on MFMA, with their FP32 operands split into BF16
// hi + lo parts), plus Adam, and the surrogate renderer with its fallback to
// the FP64 integrator.
//
// Inference (mlp_infer_rows) is row-parallel: a wave keeps its rows'
// activations in registers through all layers, and the weights come as MFMA
// fragments in a permuted order that lets one layer's accumulators serve as
// the next layer's operand directly. Training runs the forward and backward
// of every row in one kernel (train_cols), which also takes the input and
// output layers' gradient products over its rows, stores the per-sample arrays
// of the hidden layers tile-major for the hidden layers' gradient products
// (train_dw), and one more kernel (finish_step) adds every partial sum in a
// fixed order and applies Adam.
//
// Parameters: one flat FP32 vector, per layer W[out][in] then b[out] (the FP32
// master copy); the BF16 copies and fragment arrays derived from it are
// refreshed after every update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kgrt.h"
#include "kgrt_device.hpp"
#include "kgrt_mino.hpp"

namespace mlpk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kIn = 4, kH = 256, kOut = 5;
// offsets into the flat parameter vector
constexpr int64_t kW1 = 0, kB1 = kW1 + kH * kIn;
constexpr int64_t kW2 = kB1 + kH, kB2 = kW2 + kH * kH;
constexpr int64_t kW3 = kB2 + kH, kB3 = kW3 + kH * kH;
constexpr int64_t kW4 = kB3 + kH, kB4 = kW4 + kH * kH;
constexpr int64_t kW5 = kB4 + kH, kB5 = kW5 + kOut * kH;
constexpr int64_t kNumParams = kB5 + kOut;  // 199941
// Inference folds the base-2 exponential's scale c = log2(e) into the weights:
// with W1, b1..b4 scaled by -c and W5 by -1/c, every hidden layer computes
// ht = -c SiLU(z) directly from zt = -c z as zt / (1 + 2^zt) (W2..W4 are
// unchanged, since -c cancels between consecutive layers). The scaled FP32
// biases [4][256] live in a small buffer Pi, the scaled W1 and W5 in the
// inference kernel's fragment array.
constexpr float kLog2e = 1.4426950408889634f;
constexpr int64_t kPiB = 0, kPiSize = 4 * kH;
constexpr float kWCap = 1.0f, kWLogR = 10.0f, kWG = 10.0f, kWPhi = 1.0f;

// sigmoid with the hardware base-2 exponential and reciprocal (about 1 ulp
// each): plenty for BF16 activations, and no IEEE division sequence.
__device__ __forceinline__ float sigmoidf_(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// ------------------------------------------- row-parallel fused inference
// Each wave owns 16 RB rows and computes every unit of every layer for them,
// so a layer's activations never leave the wave's registers: the MFMA result
// of a 16-unit block (lane (r, g) holds units 4g..4g+3 of row r) is, after
// SiLU and conversion to BF16, directly a quarter of the next layer's B
// operand, provided the next layer's weights are stored with their inputs
// permuted to match. For k step s (units 32s..32s+31) lane group g holds
// units 32s+4g..32s+4g+3 and 32s+16+4g..32s+16+4g+3, so fragment element
// e of lane (r, g) multiplies input unit kperm(s, g, e) below. The weights of
// one hidden layer (128 KB of fragments) sit in LDS, loaded by the whole block
// between layers; all waves of the block then read the same fragments.
//
// Fragment arrays in Wr (BF16, 64 lanes x 8 values = 1 KB per fragment):
//   hidden layers l = 0..2 (W2..W4): [l][jb 16][s 8][lane 64][8], element e of
//     lane (r, g): W[16 jb + r][kperm(s, g, e)];
//   input layer (scaled W1 in hi + lo parts): [jb 16][lane][8];
//   output head (scaled W5, hi and lo parts): [s 8][part 2][lane][8].
constexpr int64_t kWrFrag = 64 * 8;
constexpr int64_t kWrHid = 0, kWrW1 = 3 * 16 * 8 * kWrFrag, kWrW5 = kWrW1 + 16 * kWrFrag;
constexpr int64_t kWrSize = kWrW5 + 8 * 2 * kWrFrag;
// three 16-row tiles per wave: each 1 KB fragment read from LDS feeds three products (the 8 waves
// of a block read every fragment of a layer, so LDS traffic per product falls as RB grows), at
// two waves per SIMD
constexpr int kRowsRB = 3, kRowsWaves = 8, kRowsThreads = 64 * kRowsWaves, kRowsTile = 16 * kRowsRB * kRowsWaves;

__host__ __device__ constexpr int kperm(int s, int g, int e) { return 32 * s + 4 * g + (e < 4 ? e : 12 + e); }

__global__ void __launch_bounds__(256) pack_rows(const float* __restrict__ P, __bf16* __restrict__ Wr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kWrSize; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(i % 8), lane = (int)((i / 8) % 64), r = lane % 16, g = lane / 16;
        const int64_t f = i / kWrFrag;  // fragment index
        float v = 0.0f;
        if (i < kWrW1) {
            const int l = (int)(f / 128), jb = (int)((f / 8) % 16), s = (int)(f % 8);
            const float* W = P + (l == 0 ? kW2 : (l == 1 ? kW3 : kW4));
            v = W[(16 * jb + r) * kH + kperm(s, g, e)];
        } else if (i < kWrW5) {
            // k 0..3 W1hi.xhi, 4..7 W1hi.xlo, 8..11 W1lo.xhi: lane group 0 holds W1hi twice, group 1 W1lo
            const int jb = (int)(f - kWrW1 / kWrFrag);
            const float w = -kLog2e * P[kW1 + (16 * jb + r) * kIn + (e & 3)];
            const float hi = (float)(__bf16)w;
            v = (g == 0) ? hi : ((g == 1 && e < 4) ? w - hi : 0.0f);
        } else {
            const int s = (int)((f - kWrW5 / kWrFrag) / 2), part = (int)((f - kWrW5 / kWrFrag) % 2);
            const float w = (r < kOut) ? -P[kW5 + r * kH + kperm(s, g, e)] / kLog2e : 0.0f;
            const float hi = (float)(__bf16)w;
            v = part == 0 ? hi : w - hi;
        }
        Wr[i] = (__bf16)v;
    }
}

__global__ void __launch_bounds__(kRowsThreads) __attribute__((amdgpu_waves_per_eu(kRowsWaves / 4, kRowsWaves / 4)))
mlp_infer_rows(const float* __restrict__ x, int64_t n, const float* __restrict__ P, const __bf16* __restrict__ Wr,
               const float* __restrict__ Pi, float* __restrict__ y) {
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
    constexpr int RB = kRowsRB;
    __shared__ bf16x8 wl[16 * 8 * 64];  // one hidden layer's fragments
    __shared__ f32x4 bl[4 * kH / 4];      // scaled biases b1..b4
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    auto silu = [](const f32x4& z) {  // ht = zt / (1 + 2^zt), see the scaling note above
        bf16x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (__bf16)(z[e] * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z[e])));
        return v;
    };
    auto cat = [](const bf16x4& a, const bf16x4& b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); };
    const int64_t ntiles = (n + kRowsTile - 1) / kRowsTile;
    for (int i = tid; i < kH; i += kRowsThreads) bl[i] = reinterpret_cast<const f32x4*>(Pi + kPiB)[i];
    __syncthreads();
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // Parameter pointers made opaque per tile: otherwise the compiler hoists
        // every fragment and bias load out of the tile loop, and those loop
        // invariants (hundreds of registers) spill.
        typedef const __attribute__((address_space(1))) bf16x8 GW;
        GW* Wg = (GW*)Wr;
        asm volatile("" : "+s"(Wg));
        const int64_t row0 = tile * kRowsTile + 16 * RB * wave;
        bf16x4 act[RB][16], nxt[RB][16];
        // input layer: B fragment of the features, split into hi + lo parts
        {
            bf16x8 xf[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int64_t row = row0 + 16 * rb + r;
                f32x4 xv = {0.f, 0.f, 0.f, 0.f};
                if (row < n && g <= 1) xv = *reinterpret_cast<const f32x4*>(x + row * kIn);
                bf16x8 f;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const __bf16 hi = (__bf16)xv[c];
                    f[c] = hi;
                    f[4 + c] = (g == 0) ? (__bf16)(xv[c] - (float)hi) : (__bf16)0.0f;
                }
                xf[rb] = f;
            }
#pragma unroll
            for (int jb = 0; jb < 16; ++jb) {
                const bf16x8 w1 = Wg[kWrW1 / 8 + jb * 64 + lane];
                const f32x4 b = bl[4 * jb + g];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) act[rb][jb] = silu(__builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, xf[rb], b, 0, 0, 0));
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // hidden layers W2..W4 from LDS
#pragma unroll 1
        for (int l = 0; l < 3; ++l) {
            __syncthreads();  // every wave is done with the previous layer's fragments
            GW* src = Wg + kWrHid / 8 + l * (16 * 8 * 64);
#pragma unroll
            for (int i = 0; i < 16 * 8 * 64 / kRowsThreads; ++i) wl[i * kRowsThreads + tid] = src[i * kRowsThreads + tid];
            __syncthreads();
            // software pipeline: the MFMAs of unit block jb run while the SiLU of jb - 1 is computed
            f32x4 prev[RB];
#pragma unroll
            for (int jb = 0; jb <= 16; ++jb) {
                f32x4 acc[RB];
                if (jb < 16) {
                    const f32x4 b = bl[(l + 1) * (kH / 4) + 4 * jb + g];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) acc[rb] = b;
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const bf16x8 w = wl[(jb * 8 + s) * 64 + lane];
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
                            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, cat(act[rb][2 * s], act[rb][2 * s + 1]), acc[rb], 0, 0, 0);
                    }
                }
                if (jb > 0) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) nxt[rb][jb - 1] = silu(prev[rb]);
                }
                if (jb < 16) {
                    // LDS reads one k step ahead of the MFMAs that use them, SiLU VALU work between
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        __builtin_amdgcn_sched_group_barrier(0x008, RB, 0);
                        if (i < 6) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        __builtin_amdgcn_sched_group_barrier(0x002, 2 * RB, 0);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) prev[rb] = acc[rb];
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int jb = 0; jb < 16; ++jb) act[rb][jb] = nxt[rb][jb];
        }
        // output head, W5 in hi + lo parts: lane (r, g) gets outputs 4g..4g+3 of row r
        f32x4 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bf16x8 wh = Wg[kWrW5 / 8 + (2 * s) * 64 + lane], wo = Wg[kWrW5 / 8 + (2 * s + 1) * 64 + lane];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const bf16x8 hv = cat(act[rb][2 * s], act[rb][2 * s + 1]);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, hv, acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wo, hv, acc[rb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int64_t row = row0 + 16 * rb + r;
            if (row < n && g == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) y[row * kOut + e] = acc[rb][e] + P[kB5 + e];
            } else if (row < n && g == 1) {
                y[row * kOut + 4] = acc[rb][0] + P[kB5 + 4];
            }
        }
    }
}

// Per-sample arrays of the training step are stored tile-major,
// [B/16][256 units][16 rows] BF16: a 16-row tile's values for one unit are 32
// contiguous bytes, so the training pass writes a unit block of a tile (16 units)
// as 512 contiguous bytes, and the whole tile is one 8 KB block.
__device__ __forceinline__ int64_t tm_index(int u, int64_t b) { return (b >> 4) * (kH * 16) + u * 16 + (b & 15); }

// The hidden layers' gradient products dL/dW_l = sum_b dz_l[b] h_{l-1}[b]^T and
// dL/db_l = sum_b dz_l[b] (l = 2..4) over kDwParts ranges of rows per layer (train_dw),
// added up in order by finish_step.
constexpr int kDwParts = 85;
struct TrainBufs {
    __bf16* hT[3];   // h of layers 1..3
    __bf16* dzT[3];  // dL/dz of layers 2..4
};

// ------------------------------------------ fused training pass
// Forward and backward of every row in one kernel (train_cols below):
//   forward: z1 = W1 x + b1 (FP32 operands as BF16 hi + lo parts), then
//     z_l = W_l h_{l-1} + b_l (l = 2..4, BF16 x BF16, FP32 accumulation),
//     h_l = SiLU(z_l); SiLU'(z_l) (BF16) kept for the backward: layers 2 and 3
//     in global memory in the accumulator layout, layer 4 in registers; the
//     head o = W5 h4 + b5 (W5 as hi + lo), the loss and dL/do;
//   backward: dh4 = dL/do W5 (both as hi + lo), dz_l = dh_l SiLU'(z_l),
//     dh_{l-1} = dz_l W_l on MFMA with W_l^T fragments (l = 4..2), SiLU'(z1)
//     recomputed from x.
// h1..h3 and dz2..dz4 go to global memory tile-major (transposed by a product
// with the identity on MFMA, 4 rows of one unit per lane) for train_dw; the
// products of dz1 with x and of h4 with dL/do are taken here over each block of
// rows. Every sum over the batch is added in a fixed order (finish_step), so a
// step's gradient does not depend on the order blocks run in.
//
// Training fragment array Wt (BF16, 1 KB fragments, unscaled weights):
//   W1 hi + lo [jb 16][lane][8] (as the inference kernel's input layer);
//   head W5 hi, lo [s 8][part 2][lane][8]: lane (r, g) element e W5[r][kperm(s, g, e)];
//   W5^T hi, lo [jb 16][part 2][lane][8]: lane (m, 0) element e < 5 W5[e][16 jb + m];
//   backward hidden W_l^T [l 3][jb 16][s 8][lane][8]: lane (r, g) element e
//     W_{l+2}[kperm(s, g, e)][16 jb + r].
// The forward hidden fragments are the inference kernel's (Wr, unscaled).
constexpr int64_t kWtW1 = 0, kWtW5 = kWtW1 + 16 * kWrFrag, kWtW5T = kWtW5 + 16 * kWrFrag;
constexpr int64_t kWtBwd = kWtW5T + 32 * kWrFrag, kWtSize = kWtBwd + 3 * 16 * 8 * kWrFrag;

__global__ void __launch_bounds__(256) pack_train(const float* __restrict__ P, __bf16* __restrict__ Wt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kWtSize; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(i % 8), lane = (int)((i / 8) % 64), r = lane % 16, g = lane / 16;
        const int64_t f = i / kWrFrag;
        float v = 0.0f;
        if (i < kWtW5) {
            // k 0..3 W1hi.xhi, 4..7 W1hi.xlo, 8..11 W1lo.xhi: lane group 0 holds W1hi twice, group 1 W1lo
            const int jb = (int)f;
            const float w = P[kW1 + (16 * jb + r) * kIn + (e & 3)];
            const float hi = (float)(__bf16)w;
            v = (g == 0) ? hi : ((g == 1 && e < 4) ? w - hi : 0.0f);
        } else if (i < kWtW5T) {
            const int64_t ff = f - kWtW5 / kWrFrag;
            const int s = (int)(ff / 2), part = (int)(ff % 2);
            const float w = (r < kOut) ? P[kW5 + r * kH + kperm(s, g, e)] : 0.0f;
            const float hi = (float)(__bf16)w;
            v = part == 0 ? hi : w - hi;
        } else if (i < kWtBwd) {
            const int64_t ff = f - kWtW5T / kWrFrag;
            const int jb = (int)(ff / 2), part = (int)(ff % 2);
            const float w = (g == 0 && e < kOut) ? P[kW5 + e * kH + 16 * jb + r] : 0.0f;
            const float hi = (float)(__bf16)w;
            v = part == 0 ? hi : w - hi;
        } else {
            const int64_t ff = f - kWtBwd / kWrFrag;
            const int l = (int)(ff / 128), jb = (int)((ff / 8) % 16), s = (int)(ff % 8);
            const float* W = P + (l == 0 ? kW2 : (l == 1 ? kW3 : kW4));
            v = W[kperm(s, g, e) * kH + 16 * jb + r];
        }
        Wt[i] = (__bf16)v;
    }
}

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

struct TrainRowsArgs {
    const float* x;
    const int32_t* idx;
    const float* t;
    int64_t n;
    const float* P;
    const __bf16* Wr;
    const __bf16* Wt;
    __bf16* hT[3];   // h1..h3, tile-major [B/16][256][16]
    __bf16* dzT[3];  // dL/dz of layers 2..4, tile-major
    __bf16* spF[2];  // SiLU'(z) of layers 2 and 3 in the accumulator layout [B/16][jb 16][lane 64][4]
    float* gpart;    // the input and output layers' gradient partials per 128-row block (see below)
    float* lpart;    // the loss of each wave's rows over n [grid][8], added up by finish_step
    float inv_n;
};

// The input and output layers' gradients leave the training pass as partial sums over each
// 128-row block, one value per position, in the order of their products' accumulators: dL/dW1
// and dL/db1 as [block][jb 16][g 4][c 5][e 4] (c < 4: W1[u][c], c = 4: b1[u]), dL/dW5 as
// [block][jb 16][g 4][o 5][e 4] (W5[o][u]), unit u = 16 jb + 4 g + e; then dL/db5 as
// [block][8].
constexpr int64_t kGpIn = 16 * 4 * 5 * 4, kGpOut = 16 * 4 * 5 * 4, kGpB5 = 8;

// ------------------------------------------ column-parallel fused training
// Forward and backward of a block of 128 rows (8 tiles of 16) by 8 waves, wave w
// owning unit blocks 2w and 2w + 1 (32 units) of every layer: its 16 weight
// fragments of a layer sit in its registers and the layer's input activations,
// all 256 units of the block's rows, in LDS, where every wave reads them as MFMA
// B operands (one 1 KB read serves both unit blocks). Each layer's output goes
// back to LDS in the position order that makes a contiguous 16-byte read the
// permuted k-step operand of the fragments above (unit block 2s + b, lane group
// g at positions 32 s + 8 g + 4 b .. + 3), so the same fragment arrays serve the
// row-parallel inference kernel. h and dz leave for HBM tile-major (transposed
// by a product with the identity), SiLU'(z2), SiLU'(z3) in the accumulator
// layout; SiLU'(z4) stays in registers.
constexpr int kTcWaves = 8, kTcThreads = 64 * kTcWaves, kTcRows = 128, kTcPitch = 256, kTcMaxGrid = 1024;
__global__ void __launch_bounds__(kTcThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
train_cols(const TrainRowsArgs A) {
    __shared__ __align__(16) __bf16 act[2][kTcRows * kTcPitch];  // two activation buffers (2 x 66 KB)
    __shared__ __align__(16) f32x4 bl[4][kH / 4];                // b1..b4
    __shared__ __align__(16) f32x4 xs[kTcRows];                  // the block's x rows
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    auto mfma = [](bf16x8 a, bf16x8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); };
    for (int i = tid; i < kH; i += kTcThreads) {
        const int L = i / (kH / 4), q = i % (kH / 4);
        const int64_t off = (L == 0 ? kB1 : (L == 1 ? kB2 : (L == 2 ? kB3 : kB4))) + 4 * q;
        bl[L][q] = f32x4{A.P[off], A.P[off + 1], A.P[off + 2], A.P[off + 3]};
    }
    // the identity as a 16x16x16 B operand: X I with X as A lands as X^T in the accumulator layout
    bf16x4 ident;
#pragma unroll
    for (int e = 0; e < 4; ++e) ident[e] = (__bf16)((g == (r >> 2) && e == (r & 3)) ? 1.0f : 0.0f);
    auto transpose = [&](const bf16x4& v) {
        const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(v, ident, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        bf16x4 t;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (__bf16)d[e];
        return t;
    };
    typedef const __attribute__((address_space(1))) bf16x8 GW;
    float lacc = 0.0f;
    const int64_t nblk = (A.n + kTcRows - 1) / kTcRows;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        GW* Wr = (GW*)A.Wr;
        GW* Wt = (GW*)A.Wt;
        const float* Pp = A.P;
        asm volatile("" : "+s"(Wr), "+s"(Wt), "+s"(Pp));
        const int64_t row0 = blk * kTcRows;
        const int ntile = (int)std::min<int64_t>(8, (A.n - row0) / 16);  // n is a multiple of 32
        __syncthreads();  // the previous block of rows is done with LDS
        if (tid < kTcRows) {
            f32x4 xv = {0.f, 0.f, 0.f, 0.f};
            if (row0 + tid < A.n) {
                const int64_t src = A.idx ? (int64_t)A.idx[row0 + tid] : row0 + tid;
                xv = *reinterpret_cast<const f32x4*>(A.x + src * kIn);
            }
            xs[tid] = xv;
        }
        __syncthreads();
        // B operand of the input layer for tile t (hi + lo parts of x, see pack_train)
        auto xfrag = [&](int t) {
            const f32x4 xv = xs[16 * t + r];
            bf16x8 f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const __bf16 hi = (__bf16)xv[c];
                f[c] = (g <= 1) ? hi : (__bf16)0.0f;
                f[4 + c] = (g == 0) ? (__bf16)(xv[c] - (float)hi) : (__bf16)0.0f;
            }
            return f;
        };
        // LDS: the 16-byte k-step operand (tile t, step s) and the 8-byte result of unit block jb.
        // A row's 32 chunks of 16 bytes are stored with the chunk index XORed with the row's
        // index in its tile, so the 16 rows of a tile that one read instruction touches at the
        // same chunk land in different banks.
        auto ldsB = [&](const __bf16* buf, int t, int s) {
            return *reinterpret_cast<const bf16x8*>(buf + (16 * t + r) * kTcPitch + 8 * ((4 * s + g) ^ r));
        };
        auto ldsR = [&](const __bf16* buf, int t, int jb) {
            return *reinterpret_cast<const bf16x4*>(buf + (16 * t + r) * kTcPitch + 8 * ((4 * (jb >> 1) + g) ^ r) + 4 * (jb & 1));
        };
        auto ldsW = [&](__bf16* buf, int t, int jb, const bf16x4& v) {
            *reinterpret_cast<bf16x4*>(buf + (16 * t + r) * kTcPitch + 8 * ((4 * (jb >> 1) + g) ^ r) + 4 * (jb & 1)) = v;
        };
        // HBM: tile t's values of unit block jb, transposed, to a tile-major array
        auto store_t = [&](const bf16x4& v, __bf16* dst, int t, int jb) {
            const bf16x4 vt = transpose(v);
            *reinterpret_cast<bf16x4*>(dst + tm_index(16 * jb + r, row0 + 16 * t + 4 * g)) = vt;
        };
        // K = 16 B operands over the 16 rows of tile t (lane (n, g): rows 16 t + 4 g + e, column n)
        // for the input and output layers' gradient products: x as hi (columns 0..3) and lo
        // (4..7) parts and a column of ones (8); dL/do (LDS, see the head) as hi (0..4) and lo
        // (8..12) parts
        auto xcols = [&](int t) {
            bf16x4 f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const f32x4 xv = xs[16 * t + 4 * g + e];
                const float v = xv[r & 3];
                const __bf16 hi = (__bf16)v;
                f[e] = r < 4 ? hi : (r < 8 ? (__bf16)(v - (float)hi) : (__bf16)(r == 8 ? 1.0f : 0.0f));
            }
            return f;
        };
        auto dcols = [&](const float* dsh, int t) {
            bf16x4 f;
            const int c = r & 7;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float v = (c < kOut && r < 13) ? dsh[(16 * t + 4 * g + e) * 8 + c] : 0.0f;
                const __bf16 hi = (__bf16)v;
                f[e] = r < 8 ? hi : (__bf16)(v - (float)hi);
            }
            return f;
        };
        auto mfma16 = [](bf16x4 a, bf16x4 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); };
        auto sp_ptr = [&](__bf16* arr, int t, int jb) {
            return reinterpret_cast<bf16x4*>(arr + ((row0 + 16 * t) >> 4) * (16 * 64 * 4) + (jb * 64 + lane) * 4);
        };
        const int jb0 = 2 * wave;  // this wave's unit blocks jb0, jb0 + 1
        // ---------------- input layer: h1 = SiLU(W1 x + b1)
        {
            const bf16x8 w1[2] = {Wt[kWtW1 / 8 + jb0 * 64 + lane], Wt[kWtW1 / 8 + (jb0 + 1) * 64 + lane]};
            const f32x4 b1[2] = {bl[0][4 * jb0 + g], bl[0][4 * (jb0 + 1) + g]};
            for (int t = 0; t < ntile; ++t) {
                const bf16x8 xf = xfrag(t);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const f32x4 z = mfma(w1[u], xf, b1[u]);
                    bf16x4 h;
#pragma unroll
                    for (int e = 0; e < 4; ++e) h[e] = (__bf16)(z[e] * sigmoidf_(z[e]));
                    ldsW(act[0], t, jb0 + u, h);
                    store_t(h, A.hT[0], t, jb0 + u);
                }
            }
        }
        __syncthreads();
        // ---------------- hidden layers W2..W4: act[l % 2] -> act[(l + 1) % 2]
        bf16x4 sp4[8][2];
#pragma unroll 1
        for (int l = 0; l < 3; ++l) {
            asm volatile("" : "+s"(Wr));
            bf16x8 w[2][8];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int s = 0; s < 8; ++s) w[u][s] = Wr[kWrHid / 8 + l * (16 * 8 * 64) + ((jb0 + u) * 8 + s) * 64 + lane];
            const f32x4 bb[2] = {bl[l + 1][4 * jb0 + g], bl[l + 1][4 * (jb0 + 1) + g]};
            const __bf16* in = act[l & 1];
            __bf16* out = act[(l + 1) & 1];
            // two tiles at a time: four independent accumulator chains (ntile is even)
#pragma unroll
            for (int t0 = 0; t0 < 8; t0 += 2) {
                if (t0 >= ntile) break;
                f32x4 z[2][2] = {{bb[0], bb[1]}, {bb[0], bb[1]}};
#pragma unroll
                for (int s = 0; s < 8; ++s) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const bf16x8 b = ldsB(in, t0 + q, s);
                        z[q][0] = mfma(w[0][s], b, z[q][0]);
                        z[q][1] = mfma(w[1][s], b, z[q][1]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int t = t0 + q;
                        bf16x4 h, spv;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float sg = sigmoidf_(z[q][u][e]);
                            h[e] = (__bf16)(z[q][u][e] * sg);
                            spv[e] = (__bf16)(sg * (1.0f + z[q][u][e] * (1.0f - sg)));
                        }
                        if (l == 2) sp4[t][u] = spv;
                        else *sp_ptr(A.spF[l], t, jb0 + u) = spv;
                        ldsW(out, t, jb0 + u, h);
                        if (l < 2) store_t(h, A.hT[l + 1], t, jb0 + u);
                    }
            }
            __syncthreads();
        }
        // ---------------- head (wave w: tile w), loss, dL/do; h4 is in act[1]
        __bf16* const dfr = act[0];  // dL/do operands of the 8 tiles (hi, lo), 16 KB
        float* const dsh = reinterpret_cast<float*>(act[0] + 8 * 1024);  // dL/do [tile 8][row 16][8], 4 KB
        float* const bsh = dsh + 8 * 16 * 8;  // dL/db5 of each tile [tile 8][8]
        if (wave < ntile) {
            const int t = wave;
            f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const bf16x8 hv = ldsB(act[1], t, s);
                o = mfma(Wt[kWtW5 / 8 + (2 * s) * 64 + lane], hv, o);
                o = mfma(Wt[kWtW5 / 8 + (2 * s + 1) * 64 + lane], hv, o);
            }
            const int64_t row = row0 + 16 * t + r;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            if (g <= 1) {
                const int64_t src = A.idx ? (int64_t)A.idx[row] : row;
                const float* tt = A.t + src * 6;
                const float m = tt[5];
                if (g == 0) {
                    const float o0 = o[0] + Pp[kB5], o1 = o[1] + Pp[kB5 + 1], o2 = o[2] + Pp[kB5 + 2], o3 = o[3] + Pp[kB5 + 3];
                    const float cap = tt[0];
                    const float sp = (o0 > 0.0f) ? o0 + log1pf(__expf(-o0)) : log1pf(__expf(o0));
                    const float e1 = o1 - tt[1], e2 = o2 - tt[2], e3 = o3 - tt[3];
                    lacc += kWCap * (sp - cap * o0) + kWLogR * e1 * e1 + kWG * e2 * e2 + kWPhi * m * e3 * e3;
                    d[0] = kWCap * (sigmoidf_(o0) - cap) * A.inv_n;
                    d[1] = 2.0f * kWLogR * e1 * A.inv_n;
                    d[2] = 2.0f * kWG * e2 * A.inv_n;
                    d[3] = 2.0f * kWPhi * m * e3 * A.inv_n;
#pragma unroll
                    for (int e = 0; e < 4; ++e) dsh[(16 * t + r) * 8 + e] = d[e];
                } else {
                    const float e4 = o[0] + Pp[kB5 + 4] - tt[4];
                    lacc += kWPhi * m * e4 * e4;
                    d[0] = 2.0f * kWPhi * m * e4 * A.inv_n;
                    dsh[(16 * t + r) * 8 + 4] = d[0];
                }
            }
            // dL/db5 over the tile's rows: lanes 0 and 16 hold the sums of columns 0..3 and 4
            {
                f32x4 ds = d;
#pragma unroll
                for (int dd = 1; dd < 16; dd <<= 1)
#pragma unroll
                    for (int e = 0; e < 4; ++e) ds[e] += __shfl_xor(ds[e], dd);
                if (lane == 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) bsh[t * 8 + e] = ds[e];
                } else if (lane == 16) {
                    bsh[t * 8 + 4] = ds[0];
                }
            }
            // B operands of dh4 = dL/do W5: lane (r, 0) holds dL/do of row r (hi and lo parts)
            const float d4 = __shfl(d[0], r + 16);
            bf16x8 dhi, dlo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float v = (g == 0 && e < kOut) ? (e < 4 ? d[e] : d4) : 0.0f;
                const __bf16 hi = (__bf16)v;
                dhi[e] = hi;
                dlo[e] = (__bf16)(v - (float)hi);
            }
            reinterpret_cast<bf16x8*>(dfr)[(2 * t) * 64 + lane] = dhi;
            reinterpret_cast<bf16x8*>(dfr)[(2 * t + 1) * 64 + lane] = dlo;
        }
        __syncthreads();
        if (wave == 0 && lane < kOut) {  // dL/db5 of the block: its tiles in order
            float sb = 0.0f;
            for (int t = 0; t < ntile; ++t) sb += bsh[t * 8 + lane];
            A.gpart[nblk * (kGpIn + kGpOut) + blk * kGpB5 + lane] = sb;
        }
        // ---------------- dz4 = (dL/do W5) SiLU'(z4) -> act[1]
        {
            const bf16x8 wh[2] = {Wt[kWtW5T / 8 + (2 * jb0) * 64 + lane], Wt[kWtW5T / 8 + (2 * (jb0 + 1)) * 64 + lane]};
            const bf16x8 wo[2] = {Wt[kWtW5T / 8 + (2 * jb0 + 1) * 64 + lane], Wt[kWtW5T / 8 + (2 * (jb0 + 1) + 1) * 64 + lane]};
            // dL/dW5 over the block's rows: h4 (in act[1] until this wave writes its units of dz4
            // there) transposed against the dL/do columns
            {
                f32x4 gw5[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (t >= ntile) break;
                    const bf16x4 dc = dcols(dsh, t);
#pragma unroll
                    for (int u = 0; u < 2; ++u) gw5[u] = mfma16(transpose(ldsR(act[1], t, jb0 + u)), dc, gw5[u]);
                }
                // lane (n, g) holds column n of units 16 jb + 4 g + e: dL/do hi (n < 5) and lo
                // (n = 8..12) parts, added here
                float* gp = A.gpart + nblk * kGpIn + blk * kGpOut;
                asm volatile("" : "+s"(gp));  // the lane addresses are formed here, not kept from the loop head
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    f32x4 v = gw5[u];
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] += __shfl_down(gw5[u][e], 8);
                    if (r < kOut) *reinterpret_cast<f32x4*>(gp + (((jb0 + u) * 4 + g) * 5 + r) * 4) = v;
                }
            }
            __bf16* dz4 = A.dzT[2];
            asm volatile("" : "+s"(dz4));  // its lane addresses are formed here, not kept from the kernel's start
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (t >= ntile) break;
                const bf16x8 dhi = reinterpret_cast<const bf16x8*>(dfr)[(2 * t) * 64 + lane];
                const bf16x8 dlo = reinterpret_cast<const bf16x8*>(dfr)[(2 * t + 1) * 64 + lane];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    f32x4 h = mfma(wh[u], dhi, f32x4{0.f, 0.f, 0.f, 0.f});
                    h = mfma(wo[u], dhi, h);
                    h = mfma(wh[u], dlo, h);
                    bf16x4 dz;
#pragma unroll
                    for (int e = 0; e < 4; ++e) dz[e] = (__bf16)(h[e] * (float)sp4[t][u][e]);
                    ldsW(act[1], t, jb0 + u, dz);
                    store_t(dz, dz4, t, jb0 + u);
                }
            }
        }
        __syncthreads();
        // ---------------- backward hidden: dh_{L-1} = dz_L W_L (L = 4, 3, 2), dz_{L-1} = dh SiLU'(z_{L-1})
#pragma unroll 1
        for (int li = 2; li >= 0; --li) {
            asm volatile("" : "+s"(Wt));
            bf16x8 w[2][8];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int s = 0; s < 8; ++s) w[u][s] = Wt[kWtBwd / 8 + li * (16 * 8 * 64) + ((jb0 + u) * 8 + s) * 64 + lane];
            const __bf16* in = act[(li + 1) & 1];  // dz4 in act[1], dz3 in act[0], dz2 in act[1]
            __bf16* out = act[li & 1];
            bf16x8 w1[2];
            f32x4 b1[2];
            f32x4 gw1[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};  // dL/dW1, dL/db1
            if (li == 0) {
                w1[0] = Wt[kWtW1 / 8 + jb0 * 64 + lane];
                w1[1] = Wt[kWtW1 / 8 + (jb0 + 1) * 64 + lane];
                b1[0] = bl[0][4 * jb0 + g];
                b1[1] = bl[0][4 * (jb0 + 1) + g];
            }
#pragma unroll
            for (int t0 = 0; t0 < 8; t0 += 2) {
                if (t0 >= ntile) break;
                f32x4 hh[2][2] = {{f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}},
                                  {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}}};
#pragma unroll
                for (int s = 0; s < 8; ++s) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const bf16x8 b = ldsB(in, t0 + q, s);
                        hh[q][0] = mfma(w[0][s], b, hh[q][0]);
                        hh[q][1] = mfma(w[1][s], b, hh[q][1]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                const int t = t0 + q;
                const f32x4 (&h)[2] = hh[q];
                bf16x8 xf;
                bf16x4 xc;
                if (li == 0) {
                    xf = xfrag(t);
                    xc = xcols(t);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    bf16x4 spv;
                    if (li > 0) {
                        spv = *sp_ptr(A.spF[li - 1], t, jb0 + u);
                    } else {
                        // layer 1: SiLU'(z1) recomputed from x
                        const f32x4 z = mfma(w1[u], xf, b1[u]);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float sg = sigmoidf_(z[e]);
                            spv[e] = (__bf16)(sg * (1.0f + z[e] * (1.0f - sg)));
                        }
                    }
                    bf16x4 dz;
#pragma unroll
                    for (int e = 0; e < 4; ++e) dz[e] = (__bf16)(h[u][e] * (float)spv[e]);
                    if (li > 0) {
                        ldsW(out, t, jb0 + u, dz);
                        store_t(dz, A.dzT[li - 1], t, jb0 + u);
                    } else {
                        gw1[u] = mfma16(transpose(dz), xc, gw1[u]);
                    }
                }
                }
            }
            if (li == 0) {  // lane (n, g): column n of units 16 jb + 4 g + e, x hi (0..3), lo (4..7), ones (8)
                float* gp = A.gpart + blk * kGpIn;
                asm volatile("" : "+s"(gp));
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    f32x4 v = gw1[u];
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] += __shfl_down(gw1[u][e], 4);
                    if (r < 4 || r == 8) *reinterpret_cast<f32x4*>(gp + (((jb0 + u) * 4 + g) * 5 + (r < 4 ? r : 4)) * 4) = v;
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int dd = 32; dd > 0; dd >>= 1) lacc += __shfl_xor(lacc, dd);
    if (lane == 0) A.lpart[blockIdx.x * kTcWaves + wave] = lacc * A.inv_n;
}

// Partial dW_L and db_L over a range of 64-row tiles: block (layer L - 2, part j) takes tiles
// [ntiles j / kDwParts, ntiles (j + 1) / kDwParts) and the whole 256 x 256 output; wave w
// holds output units 128 (w / 4) .. + 127 against input units 64 (w % 4) .. + 63 (8 x 4
// MFMA blocks). A k step is one tile, taken as two products of 32 rows (hh = 0, 1): lane
// (m, kg) of a fragment holds rows 16 kg + 8 hh .. + 7 of its unit, the same order in both
// operands, which the sum over the rows does not see. Each step's 64 fragments (dz and h of
// all 256 units, 64 KB) reach LDS by direct global-to-LDS loads, double-buffered: the next
// tile loads while the waves multiply the current one. The rows of a half-filled last tile
// (n is a multiple of 32) past n are zeroed in both operands.
constexpr int kDwWaves = 8;
__global__ void __launch_bounds__(64 * kDwWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
train_dw(const TrainBufs B, int64_t n, float* __restrict__ part) {
    __shared__ bf16x8 stg[2][64][64];  // [stage][fragment: 2 unit block + hh, dz then h][lane] (2 x 64 KB)
    const int li = blockIdx.x / kDwParts, j = blockIdx.x % kDwParts;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lg = lane >> 4;
    const int wo = wave >> 2, wk = wave & 3;  // wave-uniform (scalar registers)
    const int64_t ntiles = (n + 63) / 64;
    const int64_t t0 = ntiles * j / kDwParts, t1 = ntiles * (j + 1) / kDwParts;
    const int nsteps = (int)(t1 - t0);
    const bool tail_half = (n % 64) != 0 && t1 == ntiles;  // the last tile holds 32 valid rows
    const __bf16* dz = B.dzT[li];      // dL/dz of layer li + 2
    const __bf16* h = B.hT[li];        // h of layer li + 1
    f32x4 acc[8][4];
#pragma unroll
    for (int mi = 0; mi < 8; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = f32x4{0.f, 0.f, 0.f, 0.f};
    // dL/db_L = sum_b dz_L[b] as the product with a column of ones: wave (wo, wk) takes unit
    // blocks 2 wk and 2 wk + 1 of its 128 output units
    f32x4 bacc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (__bf16)(lr == 0 ? 1.0f : 0.0f);
    // fragments wave, wave + 8, ... of tile t0 + q into stage buf (each wave moves 8 of the 64)
    auto issue = [&](int q, int buf) {
        const int64_t tile = t0 + q;
#pragma unroll
        for (int i = 0; i < 64 / kDwWaves; ++i) {
            const int f = wave + kDwWaves * i, hh = f & 1, ub = (f >> 1) & 15;
            // rows 16 lg + 8 hh .. + 7 of the 64-row step: 16-row tile 4 tile + lg
            const __bf16* src = ((f < 32) ? dz : h) + (4 * tile + lg) * (kH * 16) + (16 * ub + lr) * 16 + 8 * hh;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                             (__attribute__((address_space(3))) void*)&stg[buf][f][0], 16, 0, 0);
        }
    };
    if (nsteps > 0) issue(0, 0);
    for (int q = 0; q < nsteps; ++q) {
        // this wave's loads of tile q are in; after the barrier every wave's are, and every wave
        // is done with the other stage
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (q + 1 < nsteps) issue(q + 1, (q + 1) & 1);
        const int buf = q & 1;
        const bool zero_hi = tail_half && q == nsteps - 1 && lg >= 2;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            bf16x8 a[8], b[4];
#pragma unroll
            for (int mi = 0; mi < 8; ++mi) a[mi] = stg[buf][(8 * wo + mi) * 2 + hh][lane];
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) b[ni] = stg[buf][32 + (4 * wk + ni) * 2 + hh][lane];
            if (zero_hi) {
#pragma unroll
                for (int mi = 0; mi < 8; ++mi) a[mi] = bf16x8{};
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) b[ni] = bf16x8{};
            }
#pragma unroll
            for (int mi = 0; mi < 8; ++mi)
#pragma unroll
                for (int ni = 0; ni < 4; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
#pragma unroll
            for (int mi = 0; mi < 8; ++mi)  // (a uniform branch: no register indexed at run time)
                if ((mi >> 1) == wk) bacc[mi & 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mi], ones, bacc[mi & 1], 0, 0, 0);
        }
    }
    // the accumulators as they are, 16 bytes per lane (dw_entry gives each one's place)
    f32x4* out = reinterpret_cast<f32x4*>(part + (int64_t)(li * kDwParts + j) * kH * kH) + wave * 32 * 64;
#pragma unroll
    for (int mi = 0; mi < 8; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) out[(mi * 4 + ni) * 64 + lane] = acc[mi][ni];
    // bias parts after the weight parts: [layer][part][256]; column 0 of the products
    if (lr == 0) {
        float* bo = part + (int64_t)3 * kDwParts * kH * kH + (int64_t)(li * kDwParts + j) * kH;
#pragma unroll
        for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
            for (int e = 0; e < 4; ++e) bo[128 * wo + 16 * (2 * wk + q2) + 4 * lg + e] = bacc[q2][e];
    }
}

// What train_dw leaves in slot j of a part: j = (((wave 8 + mi) 4 + ni) 64 + lane) 4 + e holds
// dL/dW[o][k] for output unit o = 128 (wave / 4) + 16 mi + 4 (lane / 16) + e and input unit
// k = 64 (wave % 4) + 16 ni + lane % 16; returns o kH + k.
__device__ __forceinline__ int dw_entry(int j) {
    const int e = j % 4, lane = (j / 4) % 64, t = j / 256, ni = t % 4, mi = (t / 4) % 8, wave = t / 32;
    return (128 * (wave / 4) + 16 * mi + 4 * (lane / 16) + e) * kH + 64 * (wave % 4) + 16 * ni + lane % 16;
}

// ------------------------------------------------- finishing a step
// One launch takes every gradient value from its partial sums in a fixed order: the hidden
// layers' weights and biases over train_dw's kDwParts parts (one thread per value, adding the
// parts in order), the input and output layers' over the training pass's 128-row blocks (16
// threads per value, each adding every 16th block in order, then the 16 sums in order), and the
// loss
// over the training pass's per-wave partials (the last block). For a training step the thread
// holding a gradient then applies Adam to its parameter (Kingma & Ba 2015:
// m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)) and writes the new value into
// every fragment slot that holds it: the slots pack_rows, pack_train and pack_biases fill,
// whose all-zero slots never change, so no repacking pass follows.
struct FinishArgs {
    const float* part;   // train_dw's partial sums
    const float* gpart;  // the training pass's input- and output-layer partial sums
    int64_t nrb;         // its 128-row blocks
    const float* lpart;  // the training pass's per-wave loss partials
    int nlp;
    float* loss;
    float* G;
    int adam;  // 0: gradients and loss only
    float *P, *M, *V, *Pi;
    __bf16 *Wr, *Wt;
    float lr, b1, b2, eps, c1, c2;
};
constexpr int kFinHidVals = 3 * kH * kH + 3 * kH;
constexpr int kFinHidBlocks = kFinHidVals / 256;
static_assert(kFinHidVals % 256 == 0, "one thread per hidden-layer gradient value");
constexpr int kFinSmBlocks = (kGpIn + kGpOut) / 16 + 1;
constexpr int kFinBlocks = kFinHidBlocks + kFinSmBlocks + 1;

// input unit k of a layer -> (k step s, lane group g, element e) with kperm(s, g, e) = k
__device__ __forceinline__ void kperm_inv(int k, int& s, int& g, int& e) {
    s = k >> 5;
    const int w = k & 31;
    g = (w & 15) >> 2;
    e = (w & 3) + ((w >> 4) << 2);
}

__device__ __forceinline__ void split_hi_lo(float w, __bf16& hi, __bf16& lo) {
    hi = (__bf16)w;
    lo = (__bf16)(w - (float)hi);
}

// The new value p of parameter i into its fragment slots (the layouts above pack_rows and
// pack_train, read backwards); b5 has none, the head reads it from P.
__device__ void scatter_param(const FinishArgs& F, int64_t i, float p) {
    __bf16 hi, lo;
    if (i < kB1) {  // W1[u][c]: lane group 0 holds hi at elements c and c + 4, lane group 1 lo at c
        const int u = (int)(i / kIn), c = (int)(i % kIn), r = u % 16;
        __bf16* wr = F.Wr + kWrW1 + (int64_t)(u / 16) * kWrFrag;
        __bf16* wt = F.Wt + kWtW1 + (int64_t)(u / 16) * kWrFrag;
        split_hi_lo(-kLog2e * p, hi, lo);
        wr[r * 8 + c] = hi;
        wr[r * 8 + c + 4] = hi;
        wr[(16 + r) * 8 + c] = lo;
        split_hi_lo(p, hi, lo);
        wt[r * 8 + c] = hi;
        wt[r * 8 + c + 4] = hi;
        wt[(16 + r) * 8 + c] = lo;
    } else if (i < kW2) {
        F.Pi[kPiB + (i - kB1)] = -kLog2e * p;
    } else if (i < kW5) {
        const int64_t off = i - kW2;
        const int l = (int)(off / (kH * kH + kH)), j = (int)(off % (kH * kH + kH));
        if (j >= kH * kH) {
            F.Pi[kPiB + (l + 1) * kH + (j - kH * kH)] = -kLog2e * p;
            return;
        }
        const int o = j / kH, k = j % kH;
        int s, g, e;
        kperm_inv(k, s, g, e);  // forward fragment: row o, input k
        F.Wr[kWrHid + ((int64_t)(l * 16 + o / 16) * 8 + s) * kWrFrag + (16 * g + o % 16) * 8 + e] = (__bf16)p;
        kperm_inv(o, s, g, e);  // transposed fragment: row k, input o
        F.Wt[kWtBwd + ((int64_t)(l * 16 + k / 16) * 8 + s) * kWrFrag + (16 * g + k % 16) * 8 + e] = (__bf16)p;
    } else if (i < kB5) {
        const int o = (int)((i - kW5) / kH), k = (int)((i - kW5) % kH);
        int s, g, e;
        kperm_inv(k, s, g, e);
        const int lane = 16 * g + o;
        split_hi_lo(-p / kLog2e, hi, lo);
        F.Wr[kWrW5 + (2 * s) * kWrFrag + lane * 8 + e] = hi;
        F.Wr[kWrW5 + (2 * s + 1) * kWrFrag + lane * 8 + e] = lo;
        split_hi_lo(p, hi, lo);
        F.Wt[kWtW5 + (2 * s) * kWrFrag + lane * 8 + e] = hi;
        F.Wt[kWtW5 + (2 * s + 1) * kWrFrag + lane * 8 + e] = lo;
        F.Wt[kWtW5T + (2 * (k / 16)) * kWrFrag + (k % 16) * 8 + o] = hi;
        F.Wt[kWtW5T + (2 * (k / 16) + 1) * kWrFrag + (k % 16) * 8 + o] = lo;
    }
}

__device__ __forceinline__ void finish_param(const FinishArgs& F, int64_t i, float g) {
    F.G[i] = g;
    if (!F.adam) return;
    const float m = F.b1 * F.M[i] + (1.0f - F.b1) * g;
    const float v = F.b2 * F.V[i] + (1.0f - F.b2) * g * g;
    F.M[i] = m;
    F.V[i] = v;
    const float p = F.P[i] - F.lr * (m / F.c1) / (sqrtf(v / F.c2) + F.eps);
    F.P[i] = p;
    scatter_param(F, i, p);
}

__global__ void __launch_bounds__(256) finish_step(const FinishArgs F) {
    const int tid = threadIdx.x;
    if (blockIdx.x < kFinHidBlocks) {
        const int i = blockIdx.x * 256 + tid;
        float s = 0.0f;
        if (i >= 3 * kH * kH) {  // dL/db2..b4
            const int li = (i - 3 * kH * kH) / kH, o = (i - 3 * kH * kH) % kH;
            const float* p = F.part + (int64_t)3 * kDwParts * kH * kH + (int64_t)li * kDwParts * kH + o;
#pragma unroll 17
            for (int c = 0; c < kDwParts; ++c) s += p[(int64_t)c * kH];
            finish_param(F, (li == 0 ? kB2 : (li == 1 ? kB3 : kB4)) + o, s);
        } else {
            const int li = i / (kH * kH), j = i % (kH * kH);
            const float* p = F.part + (int64_t)li * kDwParts * kH * kH + j;
#pragma unroll 17
            for (int c = 0; c < kDwParts; ++c) s += p[(int64_t)c * kH * kH];
            finish_param(F, (li == 0 ? kW2 : (li == 1 ? kW3 : kW4)) + dw_entry(j), s);
        }
        return;
    }
    if (blockIdx.x < kFinHidBlocks + kFinSmBlocks) {  // dL/db1, W1, W5, b5
        // 16 consecutive positions of one region, 16 threads each: thread k adds the blocks
        // k, k + 16, ... in order, then the 16 sums are added in order through LDS
        __shared__ float red[16][16];
        const int sb = blockIdx.x - kFinHidBlocks, q = tid & 15, k = tid >> 4;
        const int region = sb < kGpIn / 16 ? 0 : (sb < (kGpIn + kGpOut) / 16 ? 1 : 2);
        const int pos = (sb - (region == 0 ? 0 : (region == 1 ? kGpIn / 16 : (kGpIn + kGpOut) / 16))) * 16 + q;
        const int64_t stride = region == 0 ? kGpIn : (region == 1 ? kGpOut : kGpB5);
        const float* p = F.gpart + (region == 0 ? 0 : (region == 1 ? F.nrb * kGpIn : F.nrb * (kGpIn + kGpOut))) + pos;
        const bool live = pos < stride;
        float s = 0.0f;
        if (live) {
            int64_t b = k;
            for (; b + 48 < F.nrb; b += 64) {
                const float v0 = p[b * stride], v1 = p[(b + 16) * stride], v2 = p[(b + 32) * stride], v3 = p[(b + 48) * stride];
                s += v0;
                s += v1;
                s += v2;
                s += v3;
            }
            for (; b < F.nrb; b += 16) s += p[b * stride];
        }
        red[k][q] = s;
        __syncthreads();
        if (k == 0 && live) {
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < 16; ++j) v += red[j][q];
            int64_t dst;
            if (region == 2) {
                if (pos >= kOut) return;
                dst = kB5 + pos;
            } else {
                const int e = pos & 3, c = (pos >> 2) % 5, jg = pos / 20, u = 4 * jg + e;  // jg = 4 jb + g
                dst = region == 0 ? (c < 4 ? kW1 + u * kIn + c : kB1 + u) : kW5 + c * kH + u;
            }
            finish_param(F, dst, v);
        }
        return;
    }
    // the loss: thread t adds partials t, t + 256, ... in order, then a fixed tree
    __shared__ float red[4];
    float s = 0.0f;
    for (int c = tid; c < F.nlp; c += 256) s += F.lpart[c];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) s += __shfl_xor(s, d);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) *F.loss = (red[0] + red[1]) + (red[2] + red[3]);
}

// The inference kernel's scaled biases Pi (see the scaling note above).
__global__ void __launch_bounds__(256) pack_biases(const float* __restrict__ P, float* __restrict__ Pi) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kPiSize; i += gridDim.x * blockDim.x) {
        const int layer = (i - kPiB) / kH, u = (i - kPiB) % kH;
        const int64_t off = layer == 0 ? kB1 : (layer == 1 ? kB2 : (layer == 2 ? kB3 : kB4));
        Pi[i] = -kLog2e * P[off + u];
    }
}

__global__ void fill_f32(float* p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------- feature/targets
// Features of a ray (a, inclination, x, y): (a, cos(incl), x/15, y/15).
__global__ void features_kernel(const double* __restrict__ rays4, int64_t n, float* __restrict__ f) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double* q = rays4 + 4 * i;
        f[4 * i + 0] = (float)q[0];
        f[4 * i + 1] = (float)cos(q[1] * 3.14159265358979323846 / 180.0);
        f[4 * i + 2] = (float)(q[2] / 15.0);
        f[4 * i + 3] = (float)(q[3] / 15.0);
    }
}

// Training targets from integrator outputs: (captured, log r_c, g, sin phi_c,
// cos phi_c, phi valid). Rays without a recorded crossing get r_c = r_+ and
// g = 0 (zero intensity) and no phi target.
__global__ void targets_kernel(const double* __restrict__ rays4, const int32_t* __restrict__ status,
                               const double* __restrict__ r_cross, const double* __restrict__ g,
                               const double* __restrict__ phi, int64_t n, float* __restrict__ t) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t st = status[i];
        const bool crossed = (st & KGRT_CROSSED) != 0;
        const double a = rays4[4 * i];
        const double rplus = 1.0 + sqrt(1.0 - a * a);
        float* o = t + 6 * i;
        o[0] = (st & KGRT_CAPTURED) ? 1.0f : 0.0f;
        o[1] = (float)log(crossed ? r_cross[i] : rplus);
        o[2] = crossed ? (float)g[i] : 0.0f;
        o[3] = crossed ? (float)sin(phi[i]) : 0.0f;
        o[4] = crossed ? (float)cos(phi[i]) : 0.0f;
        o[5] = crossed ? 1.0f : 0.0f;
    }
}


// ------------------------------------------------------------- rendering
// One image of the thin-disk surrogate render: pixel features -> network ->
// decode, with rays the network is unsure of sent back to the FP64 integrator.
struct RenderImage {
    double a, incl_deg, sin_i, cos_i, r_obs, phi_obs, sin_p, cos_p, x_min, x_w, y_min, y_w, r_in, r_out, r_cap;
    int32_t nx, ny;
};
struct RenderCfg {
    float p_lo, p_hi, crit_band, edge_band, g_tol, grad_max;
};
constexpr int kCritBins = 1024;

__device__ __forceinline__ void pixel_xy(const RenderImage& im, int64_t p, double& x, double& y) {
    const int64_t i = p % im.nx, j = p / im.nx;
    x = im.x_min + ((i + 0.5) * im.x_w) / im.nx;
    y = im.y_min + ((j + 0.5) * im.y_w) / im.ny;
}

__global__ void cam_features(const RenderImage im, int64_t p0, int64_t cnt, float* __restrict__ f) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        double x, y;
        pixel_xy(im, p0 + i, x, y);
        f[4 * i + 0] = (float)im.a;
        f[4 * i + 1] = (float)im.cos_i;
        f[4 * i + 2] = (float)(x / 15.0);
        f[4 * i + 3] = (float)(y / 15.0);
    }
}

// Decode the network output and decide per ray; fallback rays are compacted
// (wave ballot + one atomic per wave) into a ray list for the integrator,
// which may collect rays of several images. `intensity` and `status` point at
// this image's first pixel, `img_off` is that pixel's index in the render's
// output arrays, `img_count` counts this image's fallback rays.
__global__ void __launch_bounds__(256) decode_kernel(const RenderImage im, int64_t p0, int64_t cnt,
                                                     const float* __restrict__ pred, const float* __restrict__ Rtab,
                                                     const RenderCfg cfg, double* __restrict__ intensity,
                                                     int32_t* __restrict__ status, int64_t img_off,
                                                     unsigned long long* __restrict__ fb_count,
                                                     int64_t* __restrict__ fb_idx, double* __restrict__ fb_rays,
                                                     unsigned long long* __restrict__ img_count) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < cnt; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < cnt;
        bool fb = false;
        double x = 0.0, y = 0.0;
        float pcap = 0.0f, rc = 0.0f, g = 0.0f;
        double gk = 0.0, rcx = -1.0;
        if (valid) {
            pixel_xy(im, p0 + i, x, y);
            const float o0 = pred[5 * i], o1 = pred[5 * i + 1], o2 = pred[5 * i + 2];
            pcap = 1.0f / (1.0f + __expf(-o0));
            rc = __expf(o1);
            g = o2;
            // distance from the predicted critical curve along the radius from the image centre
            const float rho = sqrtf((float)(x * x + y * y));
            const float u = (atan2f((float)y, (float)x) + 3.14159265f) * (kCritBins / 6.28318531f) - 0.5f;
            const float fl = floorf(u);
            int j0 = (int)fl;
            const float w = u - fl;
            j0 = ((j0 % kCritBins) + kCritBins) % kCritBins;
            const float Rc = (1.0f - w) * Rtab[j0] + w * Rtab[(j0 + 1) % kCritBins];
            // The predicted crossing radius is polished on the exact Mino-time relation of
            // the photon's constants of motion (Eqs. (7), (8), (13) from its start state;
            // kgrt_mino.hpp): -1 when that cannot be certified (the ray is integrated
            // instead), 0 when the ray never reaches the equator outside the capture radius.
            // On the Keplerian disk g is then fixed by the crossing radius and the
            // photon's conserved L_z (Eqs. (2), (8)); the g head only checks consistency.
            kgrt::State s0;
            double L = 0.0;
            const bool ok = kgrt::start_ray(im.a, im.a * im.a, im.r_obs, sqrt(im.r_obs * im.r_obs + im.a * im.a),
                                            im.sin_i, im.cos_i, im.sin_p, im.cos_p, im.phi_obs, x, y, s0, L);
            if (ok) {
                double sn, cn;
                kgrt::sincos_bounded(s0.th, &sn, &cn);
                const double Q = s0.pth * s0.pth + cn * cn * (L * L / (sn * sn) - im.a * im.a);  // Eq. (13), E^2 = 1
                const bool toward = (cn > 0.0) ? (s0.pth > 0.0) : (s0.pth < 0.0);  // mu = cos(theta) heads to 0
                rcx = kgrt_mino::crossing_radius(im.a, -L, Q, s0.r, cn, toward, im.r_cap, (double)rc);
            }
            const double rd = rcx;
            const bool near_disk = rd >= im.r_in - cfg.edge_band && rd <= im.r_out + cfg.edge_band;
            if (ok && near_disk) gk = kgrt::redshift(rd, kgrt::kPi / 2.0, im.a, im.a * im.a, -L);
            // steep predicted crossing radius toward a 4-neighbour in this segment (one
            // of the pair on or near the disk): the network smooths such features
            bool steep = false;
            if (cfg.grad_max > 0.0f) {
                const int64_t px = (p0 + i) % im.nx;
                const float lo_r = logf(fmaxf((float)im.r_in - cfg.edge_band, 1e-3f));
                const float hi_r = logf((float)im.r_out + cfg.edge_band);
                const float inv_dx = (float)(im.nx / im.x_w), inv_dy = (float)(im.ny / im.y_w);
                const bool me_near = o1 >= lo_r && o1 <= hi_r;
                auto check = [&](int64_t q, float inv_pitch) {
                    if (q < 0 || q >= cnt) return;
                    const float on = pred[5 * q + 1];
                    if ((me_near || (on >= lo_r && on <= hi_r)) && !(fabsf(on - o1) * inv_pitch <= cfg.grad_max))
                        steep = true;
                };
                if (px > 0) check(i - 1, inv_dx);
                if (px + 1 < im.nx) check(i + 1, inv_dx);
                check(i - im.nx, inv_dy);
                check(i + im.nx, inv_dy);
            }
            fb = !ok || steep || !(isfinite(o0) && isfinite(o1) && isfinite(o2)) || (pcap >= cfg.p_lo && pcap <= cfg.p_hi) ||
                 fabsf(rho - Rc) < cfg.crit_band || rcx < 0.0 || fabs(rcx - im.r_in) < cfg.edge_band ||
                 fabs(rcx - im.r_out) < cfg.edge_band ||
                 (cfg.g_tol > 0.0f && near_disk && !(fabs(gk - (double)g) <= (double)cfg.g_tol));
        }
        const uint64_t mask = __ballot(fb);
        unsigned long long slot0 = 0ull;
        if (mask) {
            const int leader = __ffsll((unsigned long long)mask) - 1;
            if (lane == leader) {
                slot0 = atomicAdd(fb_count, (unsigned long long)__popcll(mask));
                if (img_count) atomicAdd(img_count, (unsigned long long)__popcll(mask));
            }
            slot0 = __shfl(slot0, leader);
        }
        if (fb) {
            const unsigned long long slot = slot0 + (unsigned long long)__popcll(mask & lt);
            fb_idx[slot] = img_off + p0 + i;
            fb_rays[4 * slot + 0] = im.a;
            fb_rays[4 * slot + 1] = im.incl_deg;
            fb_rays[4 * slot + 2] = x;
            fb_rays[4 * slot + 3] = y;
        } else if (valid) {
            // thin disk (section 4.3): I = g^3 j(r_c), j = r^-3, on [r_in, r_out]
            const double rd = rcx;
            const bool on = (rd >= im.r_in) && (rd <= im.r_out) && (gk > 0.0);
            intensity[p0 + i] = on ? gk * gk * gk / (rd * rd * rd) : 0.0;
            if (status) status[p0 + i] = (pcap > 0.5f) ? KGRT_CAPTURED : KGRT_ESCAPED;
        }
    }
}

// Scatter the integrator's results for the ray list back to their pixels.
__global__ void composite_kernel(const unsigned long long* __restrict__ fb_count, int64_t list_cap,
                                 const int64_t* __restrict__ fb_idx, const double* __restrict__ fb_I,
                                 const int32_t* __restrict__ fb_st, double* __restrict__ intensity,
                                 int32_t* __restrict__ status, int64_t total) {
    const int64_t m = std::min<int64_t>((int64_t)*fb_count, list_cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = fb_idx[i];
        if (p < 0 || p >= total) continue;
        intensity[p] = fb_I[i];
        if (status) status[p] = fb_st[i] | KGRT_FALLBACK;
    }
}

// Per-image flux in a fixed order: block b of kFluxBlocks sums its own
// contiguous slice of the image (strided over its threads, then a fixed tree)
// into part[b]; flux_final adds the kFluxBlocks partial sums in order. The
// order of every addition depends only on the image size, so repeated renders
// give identical fluxes.
constexpr int kFluxBlocks = 128;
__global__ void __launch_bounds__(256) flux_partial(const double* __restrict__ I, int64_t n, double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = std::min<int64_t>(n, (int64_t)blockIdx.x * per), hi = std::min<int64_t>(n, lo + per);
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += I[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void flux_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        *out = s;
    }
}

__global__ void zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0ull;
}
__global__ void zero_f64(double* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

// ---------------------------------------------------- critical-curve table
// The image of the spherical photon orbits (section 4.2's shadow boundary):
// an orbit of radius r in [r1, r2] (prograde / retrograde circular photon
// orbits) has xi = L/E and eta = Q/E^2 (Bardeen 1973), seen at
// alpha = -xi / sin(i), beta^2 = eta + a^2 cos^2 i - xi^2 cot^2 i. Tabulated as
// radius from the image centre on kCritBins polar-angle bins from -pi:
// max over 2^16 + 1 orbit radii (cosine-clustered over the visible range,
// found on a 200001-point scan), empty bins filled by periodic linear
// interpolation. Host and device build the same table.
constexpr int kCritScan = 200000, kCritPts = 1 << 16;
constexpr double kPiD = 3.14159265358979323846;

__host__ __device__ inline double crit_beta2(double r, double a, double c, double s, double& xi) {
    xi = -(r * r * r - 3.0 * r * r + a * a * r + a * a) / (a * (r - 1.0));
    const double eta = r * r * r * (4.0 * a * a - r * (r - 3.0) * (r - 3.0)) / (a * a * (r - 1.0) * (r - 1.0));
    return eta + a * a * c * c - xi * xi * (c / s) * (c / s);
}

__host__ __device__ inline void crit_orbits(double a, double& r1, double& r2) {
    r1 = 2.0 * (1.0 + cos(2.0 / 3.0 * acos(-fabs(a))));
    r2 = 2.0 * (1.0 + cos(2.0 / 3.0 * acos(fabs(a))));
}

__host__ __device__ inline double crit_point_r(double lo, double hi, int k) {
    // clustered at the ends of the visible range, where beta ~ sqrt(r - r_end)
    return lo + (hi - lo) * 0.5 * (1.0 - cos(kPiD * k / kCritPts));
}

__host__ __device__ inline int crit_bin(double ang) {
    int j = (int)floor((ang + kPiD) / (2.0 * kPiD) * kCritBins);
    return j < 0 ? 0 : (j > kCritBins - 1 ? kCritBins - 1 : j);
}

constexpr int kCritImgs = 64;
struct CritArgs {
    double a[kCritImgs], incl_deg[kCritImgs];
};

// One block per image: table k goes to tabs + (k0 + blockIdx.x) * kCritBins.
__global__ void __launch_bounds__(256) crit_table_kernel(const CritArgs args, int k0, float* __restrict__ tabs) {
    __shared__ unsigned int R[kCritBins];
    __shared__ double rlo[256], rhi[256];
    const int tid = threadIdx.x;
    const double a = args.a[blockIdx.x];
    const double th = args.incl_deg[blockIdx.x] * kPiD / 180.0;
    float* out = tabs + (int64_t)(k0 + blockIdx.x) * kCritBins;
    const float r_schw = (float)sqrt(27.0);
    if (fabs(a) < 1e-9) {
        for (int j = tid; j < kCritBins; j += 256) out[j] = r_schw;
        return;
    }
    const double s = sin(th), c = cos(th);
    double r1, r2, xi;
    crit_orbits(a, r1, r2);
    double lo = r2, hi = r1;
    for (int k = tid; k <= kCritScan; k += 256) {
        const double r = r1 + (r2 - r1) * k / kCritScan;
        if (crit_beta2(r, a, c, s, xi) >= 0.0) {
            lo = fmin(lo, r);
            hi = fmax(hi, r);
        }
    }
    rlo[tid] = lo;
    rhi[tid] = hi;
    for (int j = tid; j < kCritBins; j += 256) R[j] = 0u;  // 0 marks an empty bin (radii are > 0)
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            rlo[tid] = fmin(rlo[tid], rlo[tid + w]);
            rhi[tid] = fmax(rhi[tid], rhi[tid + w]);
        }
        __syncthreads();
    }
    lo = rlo[0];
    hi = rhi[0];
    if (!(hi > lo)) {
        for (int j = tid; j < kCritBins; j += 256) out[j] = r_schw;
        return;
    }
    for (int k = tid; k <= kCritPts; k += 256) {
        const double r = crit_point_r(lo, hi, k);
        const double b2 = crit_beta2(r, a, c, s, xi);
        if (b2 < 0.0) continue;
        const double al = -xi / s, be = sqrt(b2);
        const float rad = (float)hypot(al, be);
        // positive floats order as their bit patterns
        atomicMax(&R[crit_bin(atan2(be, al))], __float_as_uint(rad));
        atomicMax(&R[crit_bin(atan2(-be, al))], __float_as_uint(rad));
    }
    __syncthreads();
    for (int j = tid; j < kCritBins; j += 256) {
        if (R[j] != 0u) {
            out[j] = __uint_as_float(R[j]);
            continue;
        }
        int ja = -1, jb = -1;
        for (int d = 1; d < kCritBins && ja < 0; ++d)
            if (R[(j - d + kCritBins) % kCritBins] != 0u) ja = (j - d + kCritBins) % kCritBins;
        for (int d = 1; d < kCritBins && jb < 0; ++d)
            if (R[(j + d) % kCritBins] != 0u) jb = (j + d) % kCritBins;
        if (ja < 0) {
            out[j] = r_schw;
            continue;
        }
        const float Ra = __uint_as_float(R[ja]), Rb = __uint_as_float(R[jb]);
        const int gap = (jb - ja + kCritBins) % kCritBins;
        const int d = (j - ja + kCritBins) % kCritBins;
        out[j] = Ra + (Rb - Ra) * (float)d / (float)(gap == 0 ? kCritBins : gap);
    }
}

}  // namespace mlpk

// =================================================================== host

using namespace mlpk;

struct kgrt_mlp {
    int device = 0;
    int64_t max_batch = 0;
    float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr;
    __bf16* Wr = nullptr;  // MFMA fragments of all layers for the row-parallel inference kernel
    __bf16* Wt = nullptr;  // fragments of the row-parallel training kernel (input layer, head, W^T)
    float* Pi = nullptr;   // scaled W1 and biases for inference
    // training arrays, BF16, 256 values per sample: tile-major, hT[l] the activations h_{l+1}
    // and dzT[l] the gradients dL/dz_{l+2} (l = 0..2); spF[l] SiLU'(z_{l+2}) (l = 0, 1) in the
    // training pass's accumulator layout
    __bf16 *hT[3] = {}, *dzT[3] = {}, *spF[2] = {};
    float* part = nullptr;   // weight- and bias-gradient partial sums [3][kDwParts][256 x 256], [3][kDwParts][256]
    float* gpart = nullptr;  // the input and output layers' partial sums per 128-row block
    float* lpart = nullptr;  // the training pass's per-wave loss partials [kTcMaxGrid][8]
    int64_t step = 0;
    // render workspace (grown on demand): features, outputs, fallback list and its integration
    float *r_feat = nullptr, *r_pred = nullptr, *r_tab = nullptr;
    double* r_part = nullptr;  // per-image flux partial sums [nimg][kFluxBlocks]
    // two fallback lists: one is integrated on the side stream while the next group of pixels
    // fills the other; an event per list marks its integration and composite done
    int64_t* r_idx[2] = {};
    int32_t* r_st[2] = {};
    double *r_rays[2] = {}, *r_I[2] = {};
    unsigned long long* r_cnt[2] = {};
    hipStream_t r_side = nullptr;
    hipEvent_t r_ev_fill = nullptr, r_ev_done[2] = {};
    kgrt_ctx* r_ctx = nullptr;  // the context of the fallback integrations (its own work queue)
    int64_t r_cap = 0, r_list_cap = 0, r_tab_cap = 0;
    std::string err;
};

namespace {

int mlp_fail(kgrt_mlp* m, int code, const std::string& msg) {
    if (m) m->err = msg;
    return code;
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};


}  // namespace

extern "C" {

int64_t kgrt_mlp_num_params(void) { return kNumParams; }

int kgrt_mlp_destroy(kgrt_mlp* m) {
    if (!m) return KGRT_OK;
    DevGuard g(m->device);
    if (m->r_side) (void)hipStreamSynchronize(m->r_side);
    void* ptrs[] = {m->P, m->M, m->V, m->G, m->Wr, m->Wt, m->Pi, m->part, m->gpart, m->lpart, m->r_feat, m->r_pred,
                    m->r_tab, m->r_part, m->r_idx[0], m->r_st[0], m->r_rays[0], m->r_I[0], m->r_cnt[0],
                    m->r_idx[1], m->r_st[1], m->r_rays[1], m->r_I[1], m->r_cnt[1],
                    m->hT[0], m->hT[1], m->hT[2], m->dzT[0], m->dzT[1], m->dzT[2], m->spF[0], m->spF[1]};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (m->r_ev_fill) (void)hipEventDestroy(m->r_ev_fill);
    for (hipEvent_t e : m->r_ev_done)
        if (e) (void)hipEventDestroy(e);
    if (m->r_side) (void)hipStreamDestroy(m->r_side);
    if (m->r_ctx) (void)kgrt_ctx_destroy(m->r_ctx);
    delete m;
    return KGRT_OK;
}

int kgrt_mlp_create(kgrt_ctx* ctx, int64_t max_batch, kgrt_mlp** out) {
    if (!ctx || !out) return KGRT_E_INVALID_ARG;
    *out = nullptr;
    if (max_batch < 16 || max_batch > (int64_t(1) << 24) || (max_batch % 16) != 0) return KGRT_E_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KGRT_E_NO_DEVICE;
    auto* m = new (std::nothrow) kgrt_mlp();
    if (!m) return KGRT_E_NOMEM;
    m->device = dev;
    m->max_batch = max_batch;
    const size_t hb = (size_t)((max_batch + 63) / 64 * 64) * kH * sizeof(__bf16);  // whole 64-row tiles
    bool ok = hipMalloc(&m->P, kNumParams * 4) == hipSuccess && hipMalloc(&m->M, kNumParams * 4) == hipSuccess &&
              hipMalloc(&m->V, kNumParams * 4) == hipSuccess && hipMalloc(&m->G, kNumParams * 4) == hipSuccess &&
              hipMalloc(&m->Wr, kWrSize * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->Wt, kWtSize * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->Pi, kPiSize * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->part, (size_t)3 * kDwParts * (kH * kH + kH) * 4) == hipSuccess &&
              hipMalloc(&m->gpart, (size_t)((max_batch + kTcRows - 1) / kTcRows) * (kGpIn + kGpOut + kGpB5) * 4) == hipSuccess &&
              hipMalloc(&m->lpart, (size_t)kTcMaxGrid * kTcWaves * 4) == hipSuccess;
    for (int l = 0; ok && l < 3; ++l) ok = hipMalloc(&m->hT[l], hb) == hipSuccess && hipMalloc(&m->dzT[l], hb) == hipSuccess;
    for (int l = 0; ok && l < 2; ++l) ok = hipMalloc(&m->spF[l], hb) == hipSuccess;
    if (!ok) {
        kgrt_mlp_destroy(m);
        return KGRT_E_NOMEM;
    }
    *out = m;
    return KGRT_OK;
}

const char* kgrt_mlp_last_error(const kgrt_mlp* m) { return m ? m->err.c_str() : ""; }

int kgrt_mlp_set_params(kgrt_mlp* m, const float* params, int64_t n) {
    if (!m || !params) return KGRT_E_INVALID_ARG;
    if (n != kNumParams) return mlp_fail(m, KGRT_E_INVALID_ARG, "parameter count mismatch");
    DevGuard g(m->device);
    if (hipMemcpy(m->P, params, kNumParams * 4, hipMemcpyHostToDevice) != hipSuccess)
        return mlp_fail(m, KGRT_E_HIP, "hipMemcpy failed");
    hipLaunchKernelGGL(fill_f32, dim3(256), dim3(256), 0, 0, m->M, kNumParams, 0.0f);
    hipLaunchKernelGGL(fill_f32, dim3(256), dim3(256), 0, 0, m->V, kNumParams, 0.0f);
    hipLaunchKernelGGL(pack_biases, dim3(4), dim3(256), 0, 0, m->P, m->Pi);
    hipLaunchKernelGGL(pack_rows, dim3(208), dim3(256), 0, 0, m->P, m->Wr);
    hipLaunchKernelGGL(pack_train, dim3(432), dim3(256), 0, 0, m->P, m->Wt);
    m->step = 0;
    if (hipDeviceSynchronize() != hipSuccess) return mlp_fail(m, KGRT_E_HIP, "set_params failed");
    return KGRT_OK;
}

int kgrt_mlp_get_params(kgrt_mlp* m, float* params, int64_t n) {
    if (!m || !params) return KGRT_E_INVALID_ARG;
    if (n != kNumParams) return mlp_fail(m, KGRT_E_INVALID_ARG, "parameter count mismatch");
    DevGuard g(m->device);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(params, m->P, kNumParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return mlp_fail(m, KGRT_E_HIP, "hipMemcpy failed");
    return KGRT_OK;
}

int kgrt_mlp_get_adam(kgrt_mlp* m, float* m_host, float* v_host, int64_t n, int64_t* step) {
    if (!m || !m_host || !v_host || !step) return KGRT_E_INVALID_ARG;
    if (n != kNumParams) return mlp_fail(m, KGRT_E_INVALID_ARG, "parameter count mismatch");
    DevGuard g(m->device);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(m_host, m->M, kNumParams * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(v_host, m->V, kNumParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return mlp_fail(m, KGRT_E_HIP, "hipMemcpy failed");
    *step = m->step;
    return KGRT_OK;
}

int kgrt_mlp_set_adam(kgrt_mlp* m, const float* m_host, const float* v_host, int64_t n, int64_t step) {
    if (!m || !m_host || !v_host) return KGRT_E_INVALID_ARG;
    if (n != kNumParams) return mlp_fail(m, KGRT_E_INVALID_ARG, "parameter count mismatch");
    if (step < 0) return mlp_fail(m, KGRT_E_INVALID_ARG, "step must be >= 0");
    for (int64_t i = 0; i < n; ++i)
        if (!(v_host[i] >= 0.0f) || !std::isfinite(m_host[i]) || !std::isfinite(v_host[i]))
            return mlp_fail(m, KGRT_E_INVALID_ARG, "moments must be finite and second moments >= 0");
    DevGuard g(m->device);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(m->M, m_host, kNumParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->V, v_host, kNumParams * 4, hipMemcpyHostToDevice) != hipSuccess)
        return mlp_fail(m, KGRT_E_HIP, "hipMemcpy failed");
    m->step = step;
    return KGRT_OK;
}

int kgrt_mlp_forward(kgrt_mlp* m, const float* x, float* y, int64_t n, void* stream) {
    if (!m) return KGRT_E_INVALID_ARG;
    if (n < 0) return mlp_fail(m, KGRT_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return KGRT_OK;
    if (!x || !y) return mlp_fail(m, KGRT_E_INVALID_ARG, "x and y must be device pointers");
    DevGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    // a persistent grid: as many resident blocks as fit, looping over 256-sample tiles
    int dev = 0, ncu = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mlp_infer_rows, kRowsThreads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int64_t ntiles = (n + kRowsTile - 1) / kRowsTile;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)ncu * per_cu));
    hipLaunchKernelGGL(mlp_infer_rows, dim3(grid), dim3(kRowsThreads), 0, st, x, n, m->P, m->Wr, m->Pi, y);
    return hipGetLastError() == hipSuccess ? KGRT_OK : mlp_fail(m, KGRT_E_HIP, "kernel launch failed");
}

// Loss and gradients of one batch (n <= max_batch samples, gathered through
// idx if not NULL). Gradients land in the internal buffer and, if grads is
// not NULL, are copied to grads (device, num_params floats).
}  // extern "C"

namespace {

// The loss and gradient of a batch (kgrt_mlp_loss_grads) and, with opt, the Adam step that
// follows (kgrt_mlp_train_step): the training pass, the hidden layers' gradient products and
// finish_step, three launches on one stream.
int loss_grads_step(kgrt_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t n, float* loss,
                    const kgrt_adam* opt, hipStream_t st) {
    if (n < 32 || n > m->max_batch || (n % 32) != 0)
        return mlp_fail(m, KGRT_E_INVALID_ARG, "need 32 <= n <= max_batch with n a multiple of 32");
    if (!x || !t || !loss) return mlp_fail(m, KGRT_E_INVALID_ARG, "x, t and loss must be device pointers");
    // per-sample arrays: h1..h3 and dL/dz of layers 2..4 tile-major, SiLU'(z) of layers 2
    // and 3 in the training pass's accumulator layout
    TrainRowsArgs ta{};
    ta.x = x;
    ta.idx = idx;
    ta.t = t;
    ta.n = n;
    ta.P = m->P;
    ta.Wr = m->Wr;
    ta.Wt = m->Wt;
    for (int l = 0; l < 3; ++l) {
        ta.hT[l] = m->hT[l];
        ta.dzT[l] = m->dzT[l];
    }
    ta.spF[0] = m->spF[0];
    ta.spF[1] = m->spF[1];
    ta.gpart = m->gpart;
    ta.lpart = m->lpart;
    ta.inv_n = 1.0f / (float)n;
    TrainBufs tb{};
    for (int l = 0; l < 3; ++l) {
        tb.hT[l] = ta.hT[l];
        tb.dzT[l] = ta.dzT[l];
    }
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = (int)std::min<int64_t>(std::min<int64_t>((n + kTcRows - 1) / kTcRows, ncu), kTcMaxGrid);
    hipLaunchKernelGGL(train_cols, dim3((unsigned)grid), dim3(kTcThreads), 0, st, ta);
    hipLaunchKernelGGL(train_dw, dim3(3 * kDwParts), dim3(64 * kDwWaves), 0, st, tb, n, m->part);
    // every gradient entry and the loss are written (not added) by finish_step
    FinishArgs fa{};
    fa.part = m->part;
    fa.gpart = m->gpart;
    fa.nrb = (n + kTcRows - 1) / kTcRows;
    fa.lpart = m->lpart;
    fa.nlp = grid * kTcWaves;
    fa.loss = loss;
    fa.G = m->G;
    fa.P = m->P;
    fa.M = m->M;
    fa.V = m->V;
    fa.Pi = m->Pi;
    fa.Wr = m->Wr;
    fa.Wt = m->Wt;
    if (opt) {
        m->step += 1;
        fa.adam = 1;
        fa.lr = opt->lr;
        fa.b1 = opt->beta1;
        fa.b2 = opt->beta2;
        fa.eps = opt->eps;
        fa.c1 = 1.0f - powf(opt->beta1, (float)m->step);
        fa.c2 = 1.0f - powf(opt->beta2, (float)m->step);
    }
    hipLaunchKernelGGL(finish_step, dim3(kFinBlocks), dim3(256), 0, st, fa);
    return hipGetLastError() == hipSuccess ? KGRT_OK : mlp_fail(m, KGRT_E_HIP, "kernel launch failed");
}

}  // namespace

extern "C" {

int kgrt_mlp_loss_grads(kgrt_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t n, float* loss,
                        float* grads, void* stream) {
    if (!m) return KGRT_E_INVALID_ARG;
    DevGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    const int rc = loss_grads_step(m, x, t, idx, n, loss, nullptr, st);
    if (rc != KGRT_OK) return rc;
    if (grads && hipMemcpyAsync(grads, m->G, kNumParams * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return mlp_fail(m, KGRT_E_HIP, "gradient copy failed");
    return KGRT_OK;
}

int kgrt_mlp_train_step(kgrt_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t n,
                        const kgrt_adam* opt, float* loss, void* stream) {
    if (!m || !opt) return KGRT_E_INVALID_ARG;
    if (!(opt->lr > 0.0f && opt->beta1 >= 0.0f && opt->beta1 < 1.0f && opt->beta2 >= 0.0f && opt->beta2 < 1.0f &&
          opt->eps > 0.0f))
        return mlp_fail(m, KGRT_E_INVALID_ARG, "invalid Adam settings");
    DevGuard g(m->device);
    return loss_grads_step(m, x, t, idx, n, loss, opt, (hipStream_t)stream);
}

int kgrt_surrogate_features(const double* rays4, int64_t n, float* features, void* stream) {
    if (n < 0) return KGRT_E_INVALID_ARG;
    if (n == 0) return KGRT_OK;
    if (!rays4 || !features) return KGRT_E_INVALID_ARG;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, rays4, n, features);
    return hipGetLastError() == hipSuccess ? KGRT_OK : KGRT_E_HIP;
}

int kgrt_surrogate_targets(const double* rays4, const int32_t* status, const double* r_cross, const double* g,
                           const double* phi_cross, int64_t n, float* targets, void* stream) {
    if (n < 0) return KGRT_E_INVALID_ARG;
    if (n == 0) return KGRT_OK;
    if (!rays4 || !status || !r_cross || !g || !phi_cross || !targets) return KGRT_E_INVALID_ARG;
    hipLaunchKernelGGL(targets_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, rays4, status, r_cross, g, phi_cross, n, targets);
    return hipGetLastError() == hipSuccess ? KGRT_OK : KGRT_E_HIP;
}

}  // extern "C"

namespace {

// Kerr critical curve (boundary of the photon-capture region, the shadow of
// section 4.2) as seen at infinity, tabulated as radius from the image centre
// versus polar angle on kCritBins bins. Spherical photon orbits of radius r_p:
//   xi  = -(r^3 - 3 r^2 + a^2 r + a^2) / (a (r - 1)),
//   eta = r^3 (4 a^2 - r (r - 3)^2) / (a^2 (r - 1)^2),
// alpha = -xi / sin(i), beta = +-sqrt(eta + a^2 cos^2 i - xi^2 cot^2 i); for a = 0
// the circle of radius sqrt(27). Image-plane pixels equal (alpha, beta) up to
// O(M / r_obs), which is far below the fallback band.
void critical_table(double a, double incl_deg, std::vector<float>& R) {
    R.assign(kCritBins, -1.0f);
    if (std::fabs(a) < 1e-9) {
        std::fill(R.begin(), R.end(), (float)std::sqrt(27.0));
        return;
    }
    const double th = incl_deg * kPiD / 180.0, s = std::sin(th), c = std::cos(th);
    double r1, r2, xi;
    crit_orbits(a, r1, r2);
    // visible part of [r1, r2]: where beta^2 >= 0
    double lo = r2, hi = r1;
    for (int k = 0; k <= kCritScan; ++k) {
        const double r = r1 + (r2 - r1) * k / kCritScan;
        if (crit_beta2(r, a, c, s, xi) >= 0.0) {
            lo = std::min(lo, r);
            hi = std::max(hi, r);
        }
    }
    if (!(hi > lo)) {
        std::fill(R.begin(), R.end(), (float)std::sqrt(27.0));
        return;
    }
    for (int k = 0; k <= kCritPts; ++k) {
        const double r = crit_point_r(lo, hi, k);
        const double b2 = crit_beta2(r, a, c, s, xi);
        if (b2 < 0.0) continue;
        const double al = -xi / s, be = std::sqrt(b2);
        const float rad = (float)std::hypot(al, be);
        for (double sg : {1.0, -1.0}) {
            const int j = crit_bin(std::atan2(sg * be, al));
            R[j] = std::max(R[j], rad);
        }
    }
    // fill empty bins by periodic linear interpolation between filled ones
    std::vector<int> filled;
    for (int j = 0; j < kCritBins; ++j)
        if (R[j] > 0.0f) filled.push_back(j);
    if (filled.empty()) {
        std::fill(R.begin(), R.end(), (float)std::sqrt(27.0));
        return;
    }
    std::vector<float> out(R);
    for (size_t q = 0; q < filled.size(); ++q) {
        const int ja = filled[q], jb = filled[(q + 1) % filled.size()];
        int gap = (jb - ja + kCritBins) % kCritBins;
        if (gap == 0) gap = kCritBins;
        for (int d = 1; d < gap; ++d) out[(ja + d) % kCritBins] = R[ja] + (R[jb] - R[ja]) * (float)d / (float)gap;
    }
    R = out;
}

// Render workspace: per-segment features and predictions (`seg` pixels) and
// the fallback ray list of one group of pixels (`list` entries).
int ensure_render_ws(kgrt_mlp* m, int64_t seg, int64_t list, int32_t nimg) {
    if (seg > m->r_cap) {
        if (hipDeviceSynchronize() != hipSuccess) return KGRT_E_HIP;
        if (m->r_feat) (void)hipFree(m->r_feat);
        if (m->r_pred) (void)hipFree(m->r_pred);
        m->r_feat = m->r_pred = nullptr;
        m->r_cap = 0;
        bool ok = hipMalloc(&m->r_feat, (size_t)seg * 4 * sizeof(float)) == hipSuccess &&
                  hipMalloc(&m->r_pred, (size_t)seg * 5 * sizeof(float)) == hipSuccess;
        if (!ok) return KGRT_E_NOMEM;
        m->r_cap = seg;
    }
    if (list > m->r_list_cap) {
        if (hipDeviceSynchronize() != hipSuccess) return KGRT_E_HIP;
        for (int b = 0; b < 2; ++b) {
            void* old[] = {m->r_idx[b], m->r_st[b], m->r_rays[b], m->r_I[b]};
            for (void* p : old)
                if (p) (void)hipFree(p);
            m->r_idx[b] = nullptr;
            m->r_st[b] = nullptr;
            m->r_rays[b] = m->r_I[b] = nullptr;
        }
        m->r_list_cap = 0;
        for (int b = 0; b < 2; ++b) {
            bool ok = hipMalloc(&m->r_idx[b], (size_t)list * sizeof(int64_t)) == hipSuccess &&
                      hipMalloc(&m->r_st[b], (size_t)list * sizeof(int32_t)) == hipSuccess &&
                      hipMalloc(&m->r_rays[b], (size_t)list * 4 * sizeof(double)) == hipSuccess &&
                      hipMalloc(&m->r_I[b], (size_t)list * sizeof(double)) == hipSuccess;
            if (!ok) return KGRT_E_NOMEM;
        }
        m->r_list_cap = list;
    }
    for (int b = 0; b < 2; ++b)
        if (!m->r_cnt[b] && hipMalloc(&m->r_cnt[b], sizeof(unsigned long long)) != hipSuccess) return KGRT_E_NOMEM;
    // default priority, not synchronised with the null stream: the events below order it
    if (!m->r_side && hipStreamCreateWithFlags(&m->r_side, hipStreamNonBlocking) != hipSuccess) return KGRT_E_HIP;
    if (!m->r_ev_fill && hipEventCreateWithFlags(&m->r_ev_fill, hipEventDisableTiming) != hipSuccess) return KGRT_E_HIP;
    for (int b = 0; b < 2; ++b)
        if (!m->r_ev_done[b] && hipEventCreateWithFlags(&m->r_ev_done[b], hipEventDisableTiming) != hipSuccess)
            return KGRT_E_HIP;
    // A fallback list holds the image's hardest rays (most of them near the critical curve):
    // lanes are refilled once 8 of a wave's are idle, which measured fastest for such lists (one
    // lane at a time spends more on refills than it saves; whole waves leave lanes idle behind
    // the wave's longest ray, which here differ widely)
    if (!m->r_ctx) {
        if (kgrt_ctx_create(m->device, &m->r_ctx) != KGRT_OK) return KGRT_E_HIP;
        const kgrt_launch L{256, 0, 8, KGRT_LAUNCH_PERSISTENT};
        if (kgrt_ctx_set_launch(m->r_ctx, &L) != KGRT_OK) return KGRT_E_HIP;
    }
    if (nimg > m->r_tab_cap) {
        if (m->r_tab) {
            if (hipDeviceSynchronize() != hipSuccess) return KGRT_E_HIP;
            (void)hipFree(m->r_tab);
        }
        if (m->r_part) (void)hipFree(m->r_part);
        m->r_tab = nullptr;
        m->r_part = nullptr;
        if (hipMalloc(&m->r_tab, (size_t)nimg * kCritBins * sizeof(float)) != hipSuccess ||
            hipMalloc(&m->r_part, (size_t)nimg * kFluxBlocks * sizeof(double)) != hipSuccess)
            return KGRT_E_NOMEM;
        m->r_tab_cap = nimg;
    }
    return KGRT_OK;
}

double isco_host(double a) {
    const double z1 = 1.0 + std::cbrt(1.0 - a * a) * (std::cbrt(1.0 + a) + std::cbrt(1.0 - a));
    const double z2 = std::sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - std::sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

}  // namespace

extern "C" {

int kgrt_critical_curve(double a, double incl_deg, float* radius_host, int32_t nbins) {
    if (!radius_host || nbins != kCritBins || !(std::fabs(a) < 1.0) || !(incl_deg > 0.0 && incl_deg < 180.0))
        return KGRT_E_INVALID_ARG;
    std::vector<float> R;
    critical_table(a, incl_deg, R);
    std::copy(R.begin(), R.end(), radius_host);
    return KGRT_OK;
}

int kgrt_surrogate_render(kgrt_ctx* ctx, kgrt_mlp* m, const kgrt_camera* cams, int32_t nimg, const kgrt_model* disk,
                          const kgrt_integrator* integ, const kgrt_fallback* fb, double* intensity, int32_t* status,
                          double* flux, unsigned long long* fallback_counts, void* stream) {
    if (!ctx || !m || !cams || !disk || !integ || !fb || !intensity) return KGRT_E_INVALID_ARG;
    if (nimg < 1) return mlp_fail(m, KGRT_E_INVALID_ARG, "nimg must be >= 1");
    if (disk->kind != KGRT_MODEL_THIN_DISK) return mlp_fail(m, KGRT_E_UNSUPPORTED, "the surrogate renders the thin disk");
    if (!(fb->p_lo >= 0.0f && fb->p_hi <= 1.0f && fb->p_lo <= fb->p_hi && fb->crit_band >= 0.0f && fb->edge_band >= 0.0f &&
          fb->g_tol >= 0.0f && fb->grad_max >= 0.0f))
        return mlp_fail(m, KGRT_E_INVALID_ARG, "invalid fallback settings");
    int64_t maxn = 0;
    for (int32_t k = 0; k < nimg; ++k) {
        const int rc = kgrt_check_args(&cams[k], disk, nullptr, 0, integ);
        if (rc != KGRT_OK) return mlp_fail(m, rc, "camera " + std::to_string(k) + " or model/integrator invalid");
        maxn = std::max<int64_t>(maxn, (int64_t)cams[k].nx * cams[k].ny);
    }
    DevGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    // Pixels of all images, concatenated, are handled in groups of at most
    // kListMax pixels; a group runs the network in segments of at most kSegMax
    // pixels and sends all its fallback rays to the integrator in one launch,
    // on a side stream, while the caller's stream goes on with the next group
    // (into the other of two fallback lists).
    constexpr int64_t kSegMax = int64_t(1) << 22, kListMax = int64_t(1) << 26;
    int64_t total = 0;
    for (int32_t k = 0; k < nimg; ++k) total += (int64_t)cams[k].nx * cams[k].ny;
    const int64_t seg_cap = std::max<int64_t>(16, std::min<int64_t>(maxn, kSegMax));
    const int64_t list_cap = std::max<int64_t>(16, std::min<int64_t>(total, kListMax));
    int rc = ensure_render_ws(m, seg_cap, list_cap, nimg);
    if (rc != KGRT_OK) return mlp_fail(m, rc, "render workspace allocation failed");
    for (int32_t k0 = 0; k0 < nimg; k0 += kCritImgs) {
        CritArgs ca{};
        const int cnt = std::min<int>(kCritImgs, nimg - k0);
        for (int q = 0; q < cnt; ++q) {
            ca.a[q] = cams[k0 + q].a;
            ca.incl_deg[q] = cams[k0 + q].incl_deg;
        }
        hipLaunchKernelGGL(crit_table_kernel, dim3(cnt), dim3(256), 0, st, ca, (int)k0, m->r_tab);
    }
    if (flux) hipLaunchKernelGGL(zero_f64, dim3(1), dim3(256), 0, st, flux, (int64_t)nimg);
    if (fallback_counts) hipLaunchKernelGGL(zero_u64, dim3(1), dim3(256), 0, st, fallback_counts, (int64_t)nimg);
    const RenderCfg cfg{fb->p_lo, fb->p_hi, fb->crit_band, fb->edge_band, fb->g_tol, fb->grad_max};
    // one ray list covers images of one observer distance and azimuth
    int cur = 0;  // the list being filled
    auto flush = [&](int64_t listed, double r_obs, double phi_obs) -> int {
        if (hipEventRecord(m->r_ev_fill, st) != hipSuccess || hipStreamWaitEvent(m->r_side, m->r_ev_fill, 0) != hipSuccess)
            return mlp_fail(m, KGRT_E_HIP, "stream ordering failed");
        kgrt_outputs o{};
        o.status = m->r_st[cur];
        o.intensity = m->r_I[cur];
        int r = kgrt_trace_rays_dev(m->r_ctx, m->r_rays[cur], (const int64_t*)m->r_cnt[cur], listed, r_obs, phi_obs,
                                    disk, nullptr, 0, integ, &o, m->r_side);
        if (r != KGRT_OK) return mlp_fail(m, r, std::string("fallback integration failed: ") + kgrt_last_error(m->r_ctx));
        const unsigned grid = (unsigned)std::min<int64_t>(4096, (listed + 255) / 256);
        hipLaunchKernelGGL(composite_kernel, dim3(grid), dim3(256), 0, m->r_side, m->r_cnt[cur], listed, m->r_idx[cur],
                           m->r_I[cur], m->r_st[cur], intensity, status, total);
        if (hipEventRecord(m->r_ev_done[cur], m->r_side) != hipSuccess) return mlp_fail(m, KGRT_E_HIP, "event failed");
        // the other list is reused once its previous integration and composite are done
        cur ^= 1;
        if (hipStreamWaitEvent(st, m->r_ev_done[cur], 0) != hipSuccess)
            return mlp_fail(m, KGRT_E_HIP, "stream ordering failed");
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, m->r_cnt[cur], (int64_t)1);
        return KGRT_OK;
    };
    int64_t off = 0, listed = 0;
    double g_robs = cams[0].r_obs, g_phi = cams[0].phi_obs_deg;
    for (int b = 0; b < 2; ++b)
        if (hipEventRecord(m->r_ev_done[b], st) != hipSuccess) return mlp_fail(m, KGRT_E_HIP, "event failed");
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, st, m->r_cnt[cur], (int64_t)1);
    for (int32_t k = 0; k < nimg; ++k) {
        const kgrt_camera& c = cams[k];
        const int64_t n = (int64_t)c.nx * c.ny;
        RenderImage im;
        const double inc = c.incl_deg * 3.14159265358979323846 / 180.0;
        const double pho = c.phi_obs_deg * 3.14159265358979323846 / 180.0;
        im.a = c.a;
        im.incl_deg = c.incl_deg;
        im.sin_i = std::sin(inc);
        im.cos_i = std::cos(inc);
        im.r_obs = c.r_obs;
        im.phi_obs = pho;
        im.sin_p = std::sin(pho);
        im.cos_p = std::cos(pho);
        im.x_min = c.x_min;
        im.x_w = c.x_max - c.x_min;
        im.y_min = c.y_min;
        im.y_w = c.y_max - c.y_min;
        im.r_in = (disk->r_in > 0.0) ? disk->r_in : isco_host(c.a);
        im.r_out = disk->r_out;
        im.r_cap = (1.0 + std::sqrt(1.0 - c.a * c.a)) * (1.0 + integ->horizon_delta);
        im.nx = c.nx;
        im.ny = c.ny;
        for (int64_t p0 = 0; p0 < n;) {
            if (listed > 0 && (listed == list_cap || c.r_obs != g_robs || c.phi_obs_deg != g_phi)) {
                if ((rc = flush(listed, g_robs, g_phi)) != KGRT_OK) return rc;
                listed = 0;
            }
            g_robs = c.r_obs;
            g_phi = c.phi_obs_deg;
            const int64_t cnt = std::min(std::min<int64_t>(seg_cap, n - p0), list_cap - listed);
            const unsigned grid = (unsigned)std::min<int64_t>(4096, (cnt + 255) / 256);
            hipLaunchKernelGGL(cam_features, dim3(grid), dim3(256), 0, st, im, p0, cnt, m->r_feat);
            rc = kgrt_mlp_forward(m, m->r_feat, m->r_pred, cnt, stream);
            if (rc != KGRT_OK) return rc;
            hipLaunchKernelGGL(decode_kernel, dim3(grid), dim3(256), 0, st, im, p0, cnt, m->r_pred,
                               m->r_tab + (size_t)k * kCritBins, cfg, intensity + off, status ? status + off : nullptr,
                               off, m->r_cnt[cur], m->r_idx[cur], m->r_rays[cur],
                               fallback_counts ? fallback_counts + k : nullptr);
            listed += cnt;
            p0 += cnt;
        }
        off += n;
    }
    if (listed > 0 && (rc = flush(listed, g_robs, g_phi)) != KGRT_OK) return rc;
    // the caller's stream continues after every integration and composite
    for (int b = 0; b < 2; ++b)
        if (hipStreamWaitEvent(st, m->r_ev_done[b], 0) != hipSuccess) return mlp_fail(m, KGRT_E_HIP, "stream ordering failed");
    if (flux) {
        off = 0;
        for (int32_t k = 0; k < nimg; ++k) {
            const int64_t n = (int64_t)cams[k].nx * cams[k].ny;
            double* part = m->r_part + (size_t)k * kFluxBlocks;
            hipLaunchKernelGGL(flux_partial, dim3(kFluxBlocks), dim3(256), 0, st, intensity + off, n, part);
            hipLaunchKernelGGL(flux_final, dim3(1), dim3(64), 0, st, part, kFluxBlocks, flux + k);
            off += n;
        }
    }
    return hipGetLastError() == hipSuccess ? KGRT_OK : mlp_fail(m, KGRT_E_HIP, "kernel launch failed");
}

}  // extern "C"
