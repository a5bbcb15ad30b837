// kgrt_mlp.hip -- the learned surrogate: a 4-256-256-256-256-5 SiLU perceptron
// trained and evaluated by hand-written kernels (BF16 MFMA with FP32
// accumulation for the three 256x256 layers, FP32 VALU for the 4-wide input
// layer and the 5-wide output head), plus Adam.
//
// Layouts. Activations are batch-major [B][256] BF16. The 256x256 products run
// as out[b][n] = sum_k A[b][k] Bt[n][k] on v_mfma_f32_16x16x32_bf16 with the
// MFMA's row index on n and its column index on b, so both operands are read
// K-contiguous and each lane's four accumulators are four consecutive n of one
// b (one 8-byte store). The weight-gradient products contract over the batch,
// so the forward and backward epilogues also write feature-major copies
// [256][B] of the layer inputs and of dL/dz.
//
// Parameters: one flat FP32 vector, per layer W[out][in] then b[out] (the FP32
// master copy); BF16 copies of W2..W4 in [out][in] (forward) and [in][out]
// (input gradients) are refreshed after every update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kgrt.h"

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
constexpr float kWCap = 1.0f, kWLogR = 10.0f, kWG = 10.0f, kWPhi = 1.0f;

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_(float z) { return z * sigmoidf_(z); }
__device__ __forceinline__ float silu_grad_(float z) {
    const float s = sigmoidf_(z);
    return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------ input layer
// h1 = SiLU(x W1^T + b1), x gathered through idx (or identity). One block of
// 256 threads (thread = hidden unit) handles 16 samples.
__global__ void __launch_bounds__(256) in_layer(const float* __restrict__ x, const int32_t* __restrict__ idx,
                                                int64_t n, const float* __restrict__ P, __bf16* __restrict__ h,
                                                __bf16* __restrict__ z_out, __bf16* __restrict__ hT, int64_t ldT) {
    const int o = threadIdx.x;
    const float w0 = P[kW1 + o * kIn + 0], w1 = P[kW1 + o * kIn + 1], w2 = P[kW1 + o * kIn + 2],
                w3 = P[kW1 + o * kIn + 3], bb = P[kB1 + o];
    const int64_t b0 = (int64_t)blockIdx.x * 16;
    for (int s = 0; s < 16; ++s) {
        const int64_t b = b0 + s;
        if (b >= n) break;
        const int64_t src = idx ? idx[b] : b;
        const float* xr = x + src * kIn;
        const float z = bb + w0 * xr[0] + w1 * xr[1] + w2 * xr[2] + w3 * xr[3];
        const float a = silu_(z);
        h[b * kH + o] = (__bf16)a;
        if (z_out) z_out[b * kH + o] = (__bf16)z;
        if (hT) hT[o * ldT + b] = (__bf16)a;
    }
}

// --------------------------------------------------------- MFMA product
// out[b][n] = sum_k A[b][k] * Bt[n][k], A: [rows][lda] BF16, Bt: [256][ldb] BF16,
// k in [k0, k0 + klen). One wave computes 16 rows x 64 columns; a block of
// four waves covers 16 rows x 256 columns. Grid: (row tiles, k chunks).
enum Epi { EPI_FWD = 0, EPI_BWD = 1, EPI_ATOMIC = 2 };

struct GemmArgs {
    const __bf16* A;
    int64_t lda;
    const __bf16* Bt;
    int64_t ldb;
    int64_t rows;   // multiple of 16 handled with bounds checks on the row side
    int64_t klen;   // reduction length per block (multiple of 32)
    int64_t kend;   // reduction stops at kend (multiple of 32)
    // epilogue
    const float* bias;       // EPI_FWD: [256]
    __bf16* h;               // EPI_FWD: activation out [rows][256]
    __bf16* zsave;           // EPI_FWD: pre-activation out (may be null)
    const __bf16* zin;       // EPI_BWD: pre-activation of this layer [rows][256]
    __bf16* dz;              // EPI_BWD: dL/dz out [rows][256]
    __bf16* outT;            // EPI_FWD / EPI_BWD: feature-major copy [256][ldT] (may be null)
    int64_t ldT;
    float* acc_out;          // EPI_ATOMIC: [rows][256] FP32, accumulated with atomics
};

template <int EPI>
__global__ void __launch_bounds__(256) gemm_bt(const GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 16;  // b rows of this tile
    const int64_t kbase = (int64_t)blockIdx.y * g.klen;
    const int n0 = wave * 64;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = lane & 15, lg = lane >> 4;  // MFMA lane coordinates
    const int64_t arow = r0 + lr;
    const bool arow_ok = arow < g.rows;
    const int64_t kstop = std::min<int64_t>(kbase + g.klen, g.kend);
    for (int64_t kk = kbase; kk < kstop; kk += 32) {
        const int64_t k = kk + 8 * lg;
        bf16x8 bfrag;  // MFMA B operand: column b = lr, rows k..k+7
        if (arow_ok) {
            bfrag = *reinterpret_cast<const bf16x8*>(g.A + arow * g.lda + k);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) bfrag[e] = (__bf16)0.0f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int n = n0 + 16 * t + lr;  // MFMA A operand: row n, k..k+7
            const bf16x8 afrag = *reinterpret_cast<const bf16x8*>(g.Bt + (int64_t)n * g.ldb + k);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag, acc[t], 0, 0, 0);
        }
    }
    // accumulator e of tile t holds out[b = r0 + lr][n = n0 + 16 t + 4 lg + e]
    const int64_t b = r0 + lr;
    if (b >= g.rows) return;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int nb = n0 + 16 * t + 4 * lg;
        if (EPI == EPI_ATOMIC) {
#pragma unroll
            for (int e = 0; e < 4; ++e) atomicAdd(&g.acc_out[b * kH + nb + e], acc[t][e]);
        } else if (EPI == EPI_FWD) {
            __bf16 hv[4], zv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = acc[t][e] + g.bias[nb + e];
                zv[e] = (__bf16)z;
                hv[e] = (__bf16)silu_(z);
            }
            __bf16* hp = g.h + b * kH + nb;
#pragma unroll
            for (int e = 0; e < 4; ++e) hp[e] = hv[e];
            if (g.zsave) {
                __bf16* zp = g.zsave + b * kH + nb;
#pragma unroll
                for (int e = 0; e < 4; ++e) zp[e] = zv[e];
            }
            if (g.outT) {
#pragma unroll
                for (int e = 0; e < 4; ++e) g.outT[(int64_t)(nb + e) * g.ldT + b] = hv[e];
            }
        } else {  // EPI_BWD: dz = (dL/dh) * SiLU'(z)
            __bf16 dv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = (float)g.zin[b * kH + nb + e];
                dv[e] = (__bf16)(acc[t][e] * silu_grad_(z));
            }
            __bf16* dp = g.dz + b * kH + nb;
#pragma unroll
            for (int e = 0; e < 4; ++e) dp[e] = dv[e];
            if (g.outT) {
#pragma unroll
                for (int e = 0; e < 4; ++e) g.outT[(int64_t)(nb + e) * g.ldT + b] = dv[e];
            }
        }
    }
}

// ------------------------------------------------------------ output head
// o = h4 W5^T + b5 in FP32 (one thread per sample). Training: also the loss
// (block-reduced, one atomic per block) and dL/do.
__global__ void __launch_bounds__(256) out_layer(const __bf16* __restrict__ h4, int64_t n, const float* __restrict__ P,
                                                 float* __restrict__ y, const float* __restrict__ t,
                                                 const int32_t* __restrict__ idx, float* __restrict__ dout,
                                                 float* __restrict__ loss, float inv_n) {
    __shared__ float red[256];
    __shared__ float w5[kOut * kH];
    for (int i = threadIdx.x; i < kOut * kH; i += blockDim.x) w5[i] = P[kW5 + i];
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (b < n) {
        float o[kOut];
#pragma unroll
        for (int j = 0; j < kOut; ++j) o[j] = P[kB5 + j];
        const bf16x8* hr = reinterpret_cast<const bf16x8*>(h4 + b * kH);
        for (int c = 0; c < kH / 8; ++c) {
            const bf16x8 v = hr[c];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float hv = (float)v[e];
#pragma unroll
                for (int j = 0; j < kOut; ++j) o[j] += w5[j * kH + 8 * c + e] * hv;
            }
        }
        if (y) {
#pragma unroll
            for (int j = 0; j < kOut; ++j) y[b * kOut + j] = o[j];
        }
        if (t) {
            const float* tr = t + (idx ? (int64_t)idx[b] : b) * 6;
            const float cap = tr[0], m = tr[5];
            const float sp = (o[0] > 0.0f) ? o[0] + log1pf(__expf(-o[0])) : log1pf(__expf(o[0]));
            const float e1 = o[1] - tr[1], e2 = o[2] - tr[2], e3 = o[3] - tr[3], e4 = o[4] - tr[4];
            l = kWCap * (sp - cap * o[0]) + kWLogR * e1 * e1 + kWG * e2 * e2 + kWPhi * m * (e3 * e3 + e4 * e4);
            float* d = dout + b * kOut;
            d[0] = kWCap * (sigmoidf_(o[0]) - cap) * inv_n;
            d[1] = 2.0f * kWLogR * e1 * inv_n;
            d[2] = 2.0f * kWG * e2 * inv_n;
            d[3] = 2.0f * kWPhi * m * e3 * inv_n;
            d[4] = 2.0f * kWPhi * m * e4 * inv_n;
        }
    }
    if (t && loss) {
        red[threadIdx.x] = l;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv_n);
    }
}

// Backward through the head: dz4 = (dout W5) * SiLU'(z4), plus dW5 += dout^T h4
// and db5 += sum dout. Block of 256 threads (thread = hidden unit) over a
// chunk of `per` samples.
__global__ void __launch_bounds__(256) head_back(const float* __restrict__ dout, const __bf16* __restrict__ h4,
                                                 const __bf16* __restrict__ z4, int64_t n, int per,
                                                 const float* __restrict__ P, __bf16* __restrict__ dz4,
                                                 __bf16* __restrict__ dz4T, int64_t ldT, float* __restrict__ G) {
    const int u = threadIdx.x;
    float w[kOut];
#pragma unroll
    for (int j = 0; j < kOut; ++j) w[j] = P[kW5 + j * kH + u];
    float gw[kOut] = {0.f, 0.f, 0.f, 0.f, 0.f}, gb[kOut] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = std::min<int64_t>(n, b0 + per);
    for (int64_t b = b0; b < b1; ++b) {
        const float* d = dout + b * kOut;
        float dh = 0.0f;
        const float hv = (float)h4[b * kH + u];
#pragma unroll
        for (int j = 0; j < kOut; ++j) {
            dh += d[j] * w[j];
            gw[j] += d[j] * hv;
            gb[j] += d[j];
        }
        const __bf16 dzv = (__bf16)(dh * silu_grad_((float)z4[b * kH + u]));
        dz4[b * kH + u] = dzv;
        dz4T[(int64_t)u * ldT + b] = dzv;
    }
#pragma unroll
    for (int j = 0; j < kOut; ++j) atomicAdd(&G[kW5 + j * kH + u], gw[j]);
    if (u == 0) {
#pragma unroll
        for (int j = 0; j < kOut; ++j) atomicAdd(&G[kB5 + j], gb[j]);
    }
}

// Bias gradient of a hidden layer: db[u] = sum_b dz[u][b] over the feature-major copy.
__global__ void __launch_bounds__(256) bias_grad(const __bf16* __restrict__ dzT, int64_t ldT, int64_t n,
                                                 float* __restrict__ gb) {
    __shared__ float red[256];
    const int u = blockIdx.x;
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < n; b += 256) s += (float)dzT[(int64_t)u * ldT + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[u] = red[0];
}

// dW1[u][c] = sum_b dz1[b][u] x[b][c] (inputs gathered through idx).
__global__ void __launch_bounds__(256) in_layer_back(const __bf16* __restrict__ dz1, const float* __restrict__ x,
                                                     const int32_t* __restrict__ idx, int64_t n, int per,
                                                     float* __restrict__ G) {
    const int u = threadIdx.x;
    float g[kIn] = {0.f, 0.f, 0.f, 0.f};
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = std::min<int64_t>(n, b0 + per);
    for (int64_t b = b0; b < b1; ++b) {
        const float d = (float)dz1[b * kH + u];
        const float* xr = x + (idx ? (int64_t)idx[b] : b) * kIn;
#pragma unroll
        for (int c = 0; c < kIn; ++c) g[c] += d * xr[c];
    }
#pragma unroll
    for (int c = 0; c < kIn; ++c) atomicAdd(&G[kW1 + u * kIn + c], g[c]);
}

// ------------------------------------------------------------------ Adam
// Kingma & Ba (2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void __launch_bounds__(256) adam(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
                                            const float* __restrict__ G, int64_t np, float lr, float b1, float b2,
                                            float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = G[i];
        const float m = b1 * M[i] + (1.0f - b1) * g;
        const float v = b2 * V[i] + (1.0f - b2) * g * g;
        M[i] = m;
        V[i] = v;
        P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    }
}

// BF16 copies of W2..W4: Wf[l][out][in] (forward) and Wb[l][in][out] (input gradients).
__global__ void __launch_bounds__(256) pack_weights(const float* __restrict__ P, __bf16* __restrict__ Wf,
                                                    __bf16* __restrict__ Wb) {
    const int l = blockIdx.y;  // 0..2 -> W2..W4
    const float* W = P + (l == 0 ? kW2 : (l == 1 ? kW3 : kW4));
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kH * kH; i += gridDim.x * blockDim.x) {
        const int o = i / kH, k = i % kH;
        const __bf16 v = (__bf16)W[i];
        Wf[(int64_t)l * kH * kH + i] = v;
        Wb[(int64_t)l * kH * kH + k * kH + o] = v;
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

}  // namespace mlpk

// =================================================================== host

using namespace mlpk;

struct kgrt_mlp {
    int device = 0;
    int64_t max_batch = 0;
    float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr;
    __bf16 *Wf = nullptr, *Wb = nullptr;
    // activations / gradients, batch-major [B][256] unless named T (feature-major [256][B])
    __bf16 *h[5] = {}, *z[5] = {}, *hT[4] = {}, *dz = nullptr, *dz2 = nullptr, *dzT = nullptr;
    float* dout = nullptr;
    int64_t step = 0;
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

void launch_gemm(int epi, const GemmArgs& a, int64_t rows, int64_t ksplit, hipStream_t st) {
    const dim3 grid((unsigned)((rows + 15) / 16), (unsigned)ksplit);
    if (epi == EPI_FWD) hipLaunchKernelGGL(gemm_bt<EPI_FWD>, grid, dim3(256), 0, st, a);
    else if (epi == EPI_BWD) hipLaunchKernelGGL(gemm_bt<EPI_BWD>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(gemm_bt<EPI_ATOMIC>, grid, dim3(256), 0, st, a);
}

// Forward pass over n <= max_batch samples. Training keeps pre-activations
// and feature-major copies of the hidden layer inputs.
void forward(kgrt_mlp* m, const float* x, const int32_t* idx, int64_t n, bool train, hipStream_t st) {
    const int64_t ldT = m->max_batch;
    hipLaunchKernelGGL(in_layer, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, st, x, idx, n, m->P, m->h[1],
                       train ? m->z[1] : nullptr, train ? m->hT[1] : nullptr, ldT);
    for (int l = 2; l <= 4; ++l) {
        GemmArgs a{};
        a.A = m->h[l - 1];
        a.lda = kH;
        a.Bt = m->Wf + (int64_t)(l - 2) * kH * kH;
        a.ldb = kH;
        a.rows = n;
        a.klen = kH;
        a.kend = kH;
        a.bias = m->P + (l == 2 ? kB2 : (l == 3 ? kB3 : kB4));
        a.h = m->h[l];
        a.zsave = train ? m->z[l] : nullptr;
        a.outT = (train && l < 4) ? m->hT[l] : nullptr;
        a.ldT = ldT;
        launch_gemm(EPI_FWD, a, n, 1, st);
    }
}

}  // namespace

extern "C" {

int64_t kgrt_mlp_num_params(void) { return kNumParams; }

int kgrt_mlp_destroy(kgrt_mlp* m) {
    if (!m) return KGRT_OK;
    DevGuard g(m->device);
    void* ptrs[] = {m->P, m->M, m->V, m->G, m->Wf, m->Wb, m->dz, m->dz2, m->dzT, m->dout,
                    m->h[1], m->h[2], m->h[3], m->h[4], m->z[1], m->z[2], m->z[3], m->z[4],
                    m->hT[1], m->hT[2], m->hT[3]};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
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
    const size_t hb = (size_t)max_batch * kH * sizeof(__bf16);
    bool ok = hipMalloc(&m->P, kNumParams * 4) == hipSuccess && hipMalloc(&m->M, kNumParams * 4) == hipSuccess &&
              hipMalloc(&m->V, kNumParams * 4) == hipSuccess && hipMalloc(&m->G, kNumParams * 4) == hipSuccess &&
              hipMalloc(&m->Wf, 3 * kH * kH * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->Wb, 3 * kH * kH * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->dout, (size_t)max_batch * kOut * 4) == hipSuccess;
    for (int l = 1; ok && l <= 4; ++l) ok = hipMalloc(&m->h[l], hb) == hipSuccess && hipMalloc(&m->z[l], hb) == hipSuccess;
    for (int l = 1; ok && l <= 3; ++l) ok = hipMalloc(&m->hT[l], hb) == hipSuccess;
    ok = ok && hipMalloc(&m->dz, hb) == hipSuccess && hipMalloc(&m->dz2, hb) == hipSuccess &&
         hipMalloc(&m->dzT, hb) == hipSuccess;
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
    hipLaunchKernelGGL(pack_weights, dim3(64, 3), dim3(256), 0, 0, m->P, m->Wf, m->Wb);
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

int kgrt_mlp_forward(kgrt_mlp* m, const float* x, float* y, int64_t n, void* stream) {
    if (!m) return KGRT_E_INVALID_ARG;
    if (n < 0) return mlp_fail(m, KGRT_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return KGRT_OK;
    if (!x || !y) return mlp_fail(m, KGRT_E_INVALID_ARG, "x and y must be device pointers");
    DevGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    for (int64_t b0 = 0; b0 < n; b0 += m->max_batch) {
        const int64_t nb = std::min<int64_t>(m->max_batch, n - b0);
        forward(m, x + b0 * kIn, nullptr, nb, false, st);
        hipLaunchKernelGGL(out_layer, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, m->h[4], nb, m->P,
                           y + b0 * kOut, nullptr, nullptr, nullptr, nullptr, 0.0f);
    }
    return hipGetLastError() == hipSuccess ? KGRT_OK : mlp_fail(m, KGRT_E_HIP, "kernel launch failed");
}

// Loss and gradients of one batch (n <= max_batch samples, gathered through
// idx if not NULL). Gradients land in the internal buffer and, if grads is
// not NULL, are copied to grads (device, num_params floats).
int kgrt_mlp_loss_grads(kgrt_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t n, float* loss,
                        float* grads, void* stream) {
    if (!m) return KGRT_E_INVALID_ARG;
    if (n < 32 || n > m->max_batch || (n % 32) != 0)
        return mlp_fail(m, KGRT_E_INVALID_ARG, "need 32 <= n <= max_batch with n a multiple of 32");
    if (!x || !t || !loss) return mlp_fail(m, KGRT_E_INVALID_ARG, "x, t and loss must be device pointers");
    DevGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t ldT = m->max_batch;
    hipLaunchKernelGGL(fill_f32, dim3(256), dim3(256), 0, st, m->G, kNumParams, 0.0f);
    hipLaunchKernelGGL(fill_f32, dim3(1), dim3(64), 0, st, loss, (int64_t)1, 0.0f);
    forward(m, x, idx, n, true, st);
    hipLaunchKernelGGL(out_layer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m->h[4], n, m->P, nullptr, t,
                       idx, m->dout, loss, 1.0f / (float)n);
    // head: dz4 (batch-major in dz, feature-major in dzT), dW5, db5
    const int per = 256;
    hipLaunchKernelGGL(head_back, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, st, m->dout, m->h[4], m->z[4],
                       n, per, m->P, m->dz, m->dzT, ldT, m->G);
    __bf16* dzc = m->dz;   // dL/dz of the current layer, batch-major
    __bf16* dzn = m->dz2;  // next (lower) layer's
    for (int l = 4; l >= 2; --l) {
        // dW_l[out][in] += sum_b dz_l[b][out] h_{l-1}[b][in]:  rows = out, A = dz_l^T, Bt = h_{l-1}^T
        const int64_t kchunk = 4096;
        const int64_t kpad = n;  // n is a multiple of 32
        {
            GemmArgs a{};
            a.A = m->dzT;
            a.lda = ldT;
            a.Bt = m->hT[l - 1];
            a.ldb = ldT;
            a.rows = kH;
            a.klen = std::min<int64_t>(kchunk, kpad);
            a.kend = n;
            a.acc_out = m->G + (l == 2 ? kW2 : (l == 3 ? kW3 : kW4));
            launch_gemm(EPI_ATOMIC, a, kH, (kpad + a.klen - 1) / a.klen, st);
        }
        hipLaunchKernelGGL(bias_grad, dim3(kH), dim3(256), 0, st, m->dzT, ldT, n,
                           m->G + (l == 2 ? kB2 : (l == 3 ? kB3 : kB4)));
        // dL/dz_{l-1} = (dz_l W_l) * SiLU'(z_{l-1}):  rows = b, A = dz_l, Bt = W_l^T ([in][out])
        GemmArgs a{};
        a.A = dzc;
        a.lda = kH;
        a.Bt = m->Wb + (int64_t)(l - 2) * kH * kH;
        a.ldb = kH;
        a.rows = n;
        a.klen = kH;
        a.kend = kH;
        a.zin = m->z[l - 1];
        a.dz = dzn;
        a.outT = m->dzT;  // overwritten after its last use above (stream order)
        a.ldT = ldT;
        launch_gemm(EPI_BWD, a, n, 1, st);
        std::swap(dzc, dzn);
    }
    // input layer: dW1, db1
    hipLaunchKernelGGL(in_layer_back, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, st, dzc, x, idx, n, per,
                       m->G);
    hipLaunchKernelGGL(bias_grad, dim3(kH), dim3(256), 0, st, m->dzT, ldT, n, m->G + kB1);
    if (grads && hipMemcpyAsync(grads, m->G, kNumParams * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return mlp_fail(m, KGRT_E_HIP, "gradient copy failed");
    return hipGetLastError() == hipSuccess ? KGRT_OK : mlp_fail(m, KGRT_E_HIP, "kernel launch failed");
}

int kgrt_mlp_train_step(kgrt_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t n,
                        const kgrt_adam* opt, float* loss, void* stream) {
    if (!m || !opt) return KGRT_E_INVALID_ARG;
    if (!(opt->lr > 0.0f && opt->beta1 >= 0.0f && opt->beta1 < 1.0f && opt->beta2 >= 0.0f && opt->beta2 < 1.0f &&
          opt->eps > 0.0f))
        return mlp_fail(m, KGRT_E_INVALID_ARG, "invalid Adam settings");
    int rc = kgrt_mlp_loss_grads(m, x, t, idx, n, loss, nullptr, stream);
    if (rc != KGRT_OK) return rc;
    DevGuard g(m->device);
    hipStream_t st = (hipStream_t)stream;
    m->step += 1;
    const float c1 = 1.0f - powf(opt->beta1, (float)m->step), c2 = 1.0f - powf(opt->beta2, (float)m->step);
    hipLaunchKernelGGL(adam, dim3(256), dim3(256), 0, st, m->P, m->M, m->V, m->G, kNumParams, opt->lr, opt->beta1,
                       opt->beta2, opt->eps, c1, c2);
    hipLaunchKernelGGL(pack_weights, dim3(64, 3), dim3(256), 0, st, m->P, m->Wf, m->Wb);
    return hipGetLastError() == hipSuccess ? KGRT_OK : mlp_fail(m, KGRT_E_HIP, "kernel launch failed");
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
