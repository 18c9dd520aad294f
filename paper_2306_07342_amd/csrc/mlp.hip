// Surrogate network: an ensemble of MLPs (24 -> 256 -> 256 -> 256 -> 10,
// GELU after each hidden layer) trained and evaluated by hand-written
// kernels on the matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16: bfloat16
// operands, FP32 accumulation).
//
// Number formats: FP32 master weights and Adam moments; every matrix product
// takes bfloat16 operands (weights, the input, hidden activations after
// GELU, back-propagated pre-activation gradients, each rounded to nearest
// even once) and accumulates in FP32.  Biases, pre-activations, the loss and
// the optimiser stay FP32.
//
// Kernels (one workgroup = 4 waves = 64 samples of one member):
//   k_mlp_fwd<TRAIN>   all four layers per sample tile, activations held in
//                      LDS; in training it keeps Z (FP32) and the transposed
//                      bf16 activations for the weight gradients, and turns
//                      the output into the MSE gradient and a loss partial;
//                      in inference it runs every member and writes the
//                      ensemble mean and spread.
//   k_mlp_bwd          back-propagation through layers 4..2 (the input
//                      gradient of layer 1 is not needed).
//   k_mlp_wgrad        dW = D^T A and db = sum D per 64x64 weight tile,
//                      reduced over the batch in a fixed order.
//   k_mlp_adam         Adam on the master weights, then the bf16 copies
//                      (row-major for the forward, transposed for backward).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vqd_internal.h"

namespace vqd {
namespace {

constexpr int kIn = 24, kH = 256, kOut = 10;
constexpr int kTM = 64;              // samples per workgroup
constexpr int kLDA = kH + 8;         // LDS row stride of activations (bf16)
constexpr int kMaxMembers = 8;
// parameter offsets within a member (row-major W[out][in], then b)
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH,
              kB3 = kW3 + kH * kH, kW4 = kB3 + kH, kB4 = kW4 + kOut * kH, kP = kB4 + kOut;
constexpr int kPS = (kP + 63) / 64 * 64;          // member stride of parameter arrays
static_assert(kP == VQD_MLP_N_PARAMS, "parameter layout");
// transposed bf16 copies used by back-propagation: WT_l[in][out]
constexpr int kT2 = 0, kT3 = kT2 + kH * kH, kT4 = kT3 + kH * kH, kT4ld = 16, kTS = kT4 + kH * kT4ld;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

__device__ inline f32x4 mma(uint4 a, uint4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// out[64 x 256] = act[64 x K] * B, where B[k][n] = Wrow[n][k] (row n of a
// row-major matrix with ld elements, k < kvalid, zero beyond).  Wave w owns
// columns [64w, 64w + 64): acc[row tile][col tile].  act is LDS (kLDA).
template <int K>
__device__ inline void gemm_64x256(const uint16_t *act, const uint16_t *__restrict__ Wrow, int ld, int kvalid,
                                   f32x4 (&acc)[4][4])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lk = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        uint4 a[4], b[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = *reinterpret_cast<const uint4 *>(act + (rt * 16 + lr) * kLDA + k0 + lk);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int n = 64 * w + 16 * ct + lr;
            b[ct] = (k0 + lk < kvalid) ? *reinterpret_cast<const uint4 *>(Wrow + (size_t)n * ld + k0 + lk)
                                       : uint4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mma(a[rt], b[ct], acc[rt][ct]);
    }
}

struct FwdArgs {
    const float *x;            // [*, 24] inputs (rows gathered through idx when set)
    const int *idx;            // optional row indices into x / y
    const float *y;            // [*, 10] targets (training)
    int B;                     // valid samples
    int Bp;                    // padded batch (multiple of 64), training buffers
    int members;
    float grad_scale;          // 2 / (B * 10)
    const uint16_t *w;         // bf16 weights [members][kPS]
    const float *theta;        // FP32 master (biases)
    // training outputs (member offset by blockIdx.y)
    float *z;                  // [members][3][Bp][256]
    uint16_t *a0t;             // [members][32][Bp]
    uint16_t *at;              // [members][3][256][Bp]  (A1..A3 transposed)
    uint16_t *d4t;             // [members][16][Bp]
    float *loss_part;          // [members][Bp / 64]
    // inference outputs
    float *mean;               // [B][10]
    float *spread;             // [B]
    float *member_out;         // optional [members][B][10]
};

// Stage the 64 x 24 input tile as bf16 into act (cols 24..31 and rows past B zero).
__device__ inline void load_input(const FwdArgs &A, int b0, uint16_t *act, uint16_t *a0t)
{
    for (int e = threadIdx.x; e < kTM * 32; e += blockDim.x) {
        const int r = e >> 5, c = e & 31, b = b0 + r;
        float v = 0.f;
        if (c < kIn && b < A.B) {
            const int src = A.idx ? A.idx[b] : b;
            v = A.x[(size_t)src * kIn + c];
        }
        const uint16_t h = f2bf(v);
        act[r * kLDA + c] = h;
        if (a0t) a0t[(size_t)c * A.Bp + b] = h;
    }
}

// One member's hidden layers: act0 (input, K = 32) -> act0 after three layers
// (ping-pong through act1).  Training keeps Z and the transposed activations.
template <bool TRAIN>
__device__ inline void hidden_layers(const FwdArgs &A, int m, int b0, uint16_t *act0, uint16_t *act1)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const uint16_t *wm = A.w + (size_t)m * kPS;
    const float *th = A.theta + (size_t)m * kPS;
    uint16_t *src = act0, *dst = act1;
    for (int layer = 0; layer < 3; ++layer) {
        f32x4 acc[4][4];
        if (layer == 0)
            gemm_64x256<32>(src, wm + kW1, kIn, kIn, acc);
        else
            gemm_64x256<kH>(src, wm + (layer == 1 ? kW2 : kW3), kH, kH, acc);
        const float *bias = th + (layer == 0 ? kB1 : layer == 1 ? kB2 : kB3);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = 64 * w + 16 * ct + lr;
            const float bv = bias[col];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                uint16_t h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rt * 16 + 4 * lq + r;
                    const float zz = acc[rt][ct][r] + bv;
                    if constexpr (TRAIN)
                        A.z[(((size_t)m * 3 + layer) * A.Bp + b0 + row) * kH + col] = zz;
                    h[r] = f2bf(gelu(zz));
                    dst[row * kLDA + col] = h[r];
                }
                if constexpr (TRAIN) {
                    uint2 pk;
                    pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                    pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                    *reinterpret_cast<uint2 *>(A.at + (((size_t)m * 3 + layer) * kH + col) * A.Bp + b0 + rt * 16 +
                                               4 * lq) = pk;
                }
            }
        }
        __syncthreads();
        uint16_t *t = src;
        src = dst;
        dst = t;
    }
    // the last activations are in src == act1 (three swaps)
}

// Output layer for the row tile of wave w: returns o[r] for rows
// 16w + 4*lq + r, column lr (valid when lr < 10).
__device__ inline f32x4 output_layer(const FwdArgs &A, int m, const uint16_t *act)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lk = 8 * (lane >> 4);
    const uint16_t *w4 = A.w + (size_t)m * kPS + kW4;
    f32x4 acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int k0 = 0; k0 < kH; k0 += 32) {
        const uint4 a = *reinterpret_cast<const uint4 *>(act + (16 * w + lr) * kLDA + k0 + lk);
        const uint4 b = (lr < kOut) ? *reinterpret_cast<const uint4 *>(w4 + (size_t)lr * kH + k0 + lk)
                                    : uint4{0u, 0u, 0u, 0u};
        acc = mma(a, b, acc);
    }
    const float bv = (lr < kOut) ? A.theta[(size_t)m * kPS + kB4 + lr] : 0.f;
    for (int r = 0; r < 4; ++r) acc[r] += bv;
    return acc;
}

__global__ void __launch_bounds__(256) k_mlp_fwd_train(FwdArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t act0[kTM * kLDA];
    __shared__ __attribute__((aligned(16))) uint16_t act1[kTM * kLDA];
    __shared__ float red[4];
    const int m = blockIdx.y, b0 = blockIdx.x * kTM;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lq = lane >> 4;
    load_input(A, b0, act0, A.a0t + (size_t)m * 32 * A.Bp);
    __syncthreads();
    hidden_layers<true>(A, m, b0, act0, act1);
    const f32x4 o = output_layer(A, m, act1);
    float sq = 0.f;
    uint16_t h[4];
    for (int r = 0; r < 4; ++r) {
        const int b = b0 + 16 * w + 4 * lq + r;
        float d = 0.f;
        if (lr < kOut && b < A.B) {
            const int src = A.idx ? A.idx[b] : b;
            d = o[r] - A.y[(size_t)src * kOut + lr];
        }
        sq += d * d;
        h[r] = f2bf(d * A.grad_scale);
    }
    uint2 pk;
    pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
    pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
    *reinterpret_cast<uint2 *>(A.d4t + ((size_t)m * 16 + lr) * A.Bp + b0 + 16 * w + 4 * lq) = pk;
    // loss partial of the tile, fixed order: lanes by shuffle tree, waves in order
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_down(sq, off, 64);
    if (lane == 0) red[w] = sq;
    __syncthreads();
    if (threadIdx.x == 0)
        A.loss_part[(size_t)m * (A.Bp / kTM) + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_mlp_predict(FwdArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t act0[kTM * kLDA];
    __shared__ __attribute__((aligned(16))) uint16_t act1[kTM * kLDA];
    __shared__ uint16_t xin[kTM * 32];
    __shared__ float outs[kMaxMembers][kTM][kOut];
    const int b0 = blockIdx.x * kTM;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lq = lane >> 4;
    load_input(A, b0, act0, nullptr);
    __syncthreads();
    for (int e = threadIdx.x; e < kTM * 32; e += blockDim.x) xin[e] = act0[(e >> 5) * kLDA + (e & 31)];
    for (int m = 0; m < A.members; ++m) {
        if (m > 0) {
            __syncthreads();
            for (int e = threadIdx.x; e < kTM * 32; e += blockDim.x) act0[(e >> 5) * kLDA + (e & 31)] = xin[e];
            __syncthreads();
        }
        hidden_layers<false>(A, m, b0, act0, act1);
        const f32x4 o = output_layer(A, m, act1);
        if (lr < kOut)
            for (int r = 0; r < 4; ++r) outs[m][16 * w + 4 * lq + r][lr] = o[r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kTM * kOut; e += blockDim.x) {
        const int r = e / kOut, c = e % kOut, b = b0 + r;
        if (b >= A.B) continue;
        float s = 0.f;
        for (int m = 0; m < A.members; ++m) s += outs[m][r][c];
        const float mu = s / (float)A.members;
        A.mean[(size_t)b * kOut + c] = mu;
        if (A.member_out)
            for (int m = 0; m < A.members; ++m) A.member_out[((size_t)m * A.B + b) * kOut + c] = outs[m][r][c];
    }
    if (threadIdx.x < kTM && b0 + (int)threadIdx.x < A.B) {
        const int r = threadIdx.x;
        float sp = 0.f;
        for (int c = 0; c < kOut; ++c) {
            float s = 0.f;
            for (int m = 0; m < A.members; ++m) s += outs[m][r][c];
            const float mu = s / (float)A.members;
            float v = 0.f;
            for (int m = 0; m < A.members; ++m) {
                const float d = outs[m][r][c] - mu;
                v += d * d;
            }
            sp = fmaxf(sp, sqrtf(v / (float)A.members));
        }
        A.spread[b0 + r] = sp;
    }
}

struct BwdArgs {
    int Bp;
    const uint16_t *wt;        // [members][kTS] transposed bf16 weights
    const float *z;            // [members][3][Bp][256]
    const uint16_t *d4t;       // [members][16][Bp]
    uint16_t *dt;              // [members][3][256][Bp]  (D1..D3 transposed)
};

__global__ void __launch_bounds__(256) k_mlp_bwd(BwdArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t d0[kTM * kLDA];
    __shared__ __attribute__((aligned(16))) uint16_t d1[kTM * kLDA];
    const int m = blockIdx.y, b0 = blockIdx.x * kTM;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lq = lane >> 4;
    // D4 tile (64 x 16, zero to 32 columns)
    for (int e = threadIdx.x; e < kTM * 32; e += blockDim.x) {
        const int c = e / kTM, r = e % kTM;
        d0[r * kLDA + c] = (c < 16) ? A.d4t[((size_t)m * 16 + c) * A.Bp + b0 + r] : (uint16_t)0;
    }
    __syncthreads();
    const uint16_t *wt = A.wt + (size_t)m * kTS;
    uint16_t *src = d0, *dst = d1;
    // layer l = 4, 3, 2: D_{l-1} = bf16((D_l W_l) * gelu'(Z_{l-1}))
    for (int step = 0; step < 3; ++step) {
        const int zl = 2 - step;                 // index of Z_{l-1} / D_{l-1}: 2, 1, 0
        f32x4 acc[4][4];
        if (step == 0)
            gemm_64x256<32>(src, wt + kT4, kT4ld, 16, acc);
        else
            gemm_64x256<kH>(src, wt + (step == 1 ? kT3 : kT2), kH, kH, acc);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = 64 * w + 16 * ct + lr;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                uint16_t h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rt * 16 + 4 * lq + r;
                    const float zz = A.z[(((size_t)m * 3 + zl) * A.Bp + b0 + row) * kH + col];
                    h[r] = f2bf(acc[rt][ct][r] * gelu_grad(zz));
                    if (step < 2) dst[row * kLDA + col] = h[r];
                }
                uint2 pk;
                pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                *reinterpret_cast<uint2 *>(A.dt + (((size_t)m * 3 + zl) * kH + col) * A.Bp + b0 + rt * 16 + 4 * lq) = pk;
            }
        }
        __syncthreads();
        uint16_t *t = src;
        src = dst;
        dst = t;
    }
}

struct WgradArgs {
    int Bp;
    const uint16_t *a0t, *at, *d4t, *dt;
    float *grad;               // [members][kPS]
};

// Weight-gradient tiles of one member: (layer, o tile, i tile), 40 in all.
__device__ inline void wgrad_tile(int t, int &layer, int &o0, int &i0)
{
    if (t < 4) { layer = 1; o0 = 64 * t; i0 = 0; return; }
    t -= 4;
    if (t < 32) { layer = 2 + t / 16; o0 = 64 * ((t % 16) / 4); i0 = 64 * (t % 4); return; }
    t -= 32;
    layer = 4; o0 = 0; i0 = 64 * t;
}
constexpr int kWgradTiles = 40;

__global__ void __launch_bounds__(256) k_mlp_wgrad(WgradArgs A)
{
    const int m = blockIdx.y;
    int layer, o0, i0;
    wgrad_tile(blockIdx.x, layer, o0, i0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lq = lane >> 4, lk = 8 * lq;
    // D_l^T rows (o) and A_{l-1}^T rows (i), each Bp long
    const uint16_t *D, *X;
    int o_rows, i_rows, O, I, offW, offB;
    switch (layer) {
    case 1: D = A.dt + ((size_t)m * 3 + 0) * kH * A.Bp; X = A.a0t + (size_t)m * 32 * A.Bp;
            o_rows = kH; i_rows = 32; O = kH; I = kIn; offW = kW1; offB = kB1; break;
    case 2: D = A.dt + ((size_t)m * 3 + 1) * kH * A.Bp; X = A.at + ((size_t)m * 3 + 0) * kH * A.Bp;
            o_rows = kH; i_rows = kH; O = kH; I = kH; offW = kW2; offB = kB2; break;
    case 3: D = A.dt + ((size_t)m * 3 + 2) * kH * A.Bp; X = A.at + ((size_t)m * 3 + 1) * kH * A.Bp;
            o_rows = kH; i_rows = kH; O = kH; I = kH; offW = kW3; offB = kB3; break;
    default: D = A.d4t + (size_t)m * 16 * A.Bp; X = A.at + ((size_t)m * 3 + 2) * kH * A.Bp;
            o_rows = 16; i_rows = kH; O = kOut; I = kH; offW = kW4; offB = kB4; break;
    }
    const int o = o0 + 16 * w + lr;            // A-operand row of this lane
    const bool o_ok = o < o_rows;
    f32x4 acc[4];
    for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < A.Bp; k0 += 32) {
        const uint4 a = o_ok ? *reinterpret_cast<const uint4 *>(D + (size_t)o * A.Bp + k0 + lk) : uint4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int i = i0 + 16 * ct + lr;
            const uint4 b = (i < i_rows) ? *reinterpret_cast<const uint4 *>(X + (size_t)i * A.Bp + k0 + lk)
                                         : uint4{0u, 0u, 0u, 0u};
            acc[ct] = mma(a, b, acc[ct]);
        }
    }
    float *g = A.grad + (size_t)m * kPS;
    for (int ct = 0; ct < 4; ++ct)
        for (int r = 0; r < 4; ++r) {
            const int oo = o0 + 16 * w + 4 * lq + r, ii = i0 + 16 * ct + lr;
            if (oo < O && ii < I) g[offW + (size_t)oo * I + ii] = acc[ct][r];
        }
    // bias gradient: the i0 == 0 tile sums its 64 rows of D over the batch
    if (i0 == 0 && threadIdx.x < 64) {
        const int oo = o0 + threadIdx.x;
        if (oo < O) {
            const uint16_t *row = D + (size_t)oo * A.Bp;
            float s = 0.f;
            for (int b = 0; b < A.Bp; b += 8) {
                const uint4 v = *reinterpret_cast<const uint4 *>(row + b);
                const uint32_t u[4] = {v.x, v.y, v.z, v.w};
                for (int j = 0; j < 4; ++j) s += bf2f(u[j] & 0xffffu) + bf2f(u[j] >> 16);
            }
            g[offB + oo] = s;
        }
    }
}

__global__ void k_mlp_loss(const float *part, int nblk, int members, float inv_count, float *loss)
{
    const int m = threadIdx.x;
    if (m >= members) return;
    float s = 0.f;
    for (int i = 0; i < nblk; ++i) s += part[(size_t)m * nblk + i];
    loss[m] = s * inv_count;
}

struct AdamArgs {
    int members;
    int apply;                 // 0: only refresh the bf16 copies
    // omb = 1 - beta, rounded once from double (1 - 0.999f would be 1.3e-5 off)
    float lr, beta1, beta2, omb1, omb2, eps, c1, c2;   // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
    float *theta, *m1, *m2;
    const float *grad;
    uint16_t *w, *wt;
};

__global__ void k_mlp_adam(AdamArgs A)
{
    const size_t n = (size_t)A.members * kP;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(e / kP), p = (int)(e % kP);
        const size_t idx = (size_t)m * kPS + p;
        float th = A.theta[idx];
        if (A.apply) {
            const float g = A.grad[idx];
            const float a = A.beta1 * A.m1[idx] + A.omb1 * g;
            const float v = A.beta2 * A.m2[idx] + A.omb2 * g * g;
            A.m1[idx] = a;
            A.m2[idx] = v;
            th -= A.lr * (a * A.c1) / (sqrtf(v * A.c2) + A.eps);
            A.theta[idx] = th;
        }
        const uint16_t h = f2bf(th);
        A.w[idx] = h;
        uint16_t *wt = A.wt + (size_t)m * kTS;
        if (p >= kW2 && p < kB2) {
            const int q = p - kW2, o = q / kH, i = q % kH;
            wt[kT2 + i * kH + o] = h;
        } else if (p >= kW3 && p < kB3) {
            const int q = p - kW3, o = q / kH, i = q % kH;
            wt[kT3 + i * kH + o] = h;
        } else if (p >= kW4 && p < kB4) {
            const int q = p - kW4, o = q / kH, i = q % kH;
            wt[kT4 + i * kT4ld + o] = h;
        }
    }
}

}  // namespace
}  // namespace vqd

using namespace vqd;

struct vqd_mlp {
    int members = 0, max_batch = 0, Bp_max = 0, device = -1;
    long long step = 0;
    float *theta = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    uint16_t *w = nullptr, *wt = nullptr;
    float *z = nullptr, *loss_part = nullptr, *loss = nullptr;
    uint16_t *a0t = nullptr, *at = nullptr, *d4t = nullptr, *dt = nullptr;
    void *block = nullptr;
};

namespace {

int mlp_alloc(vqd_mlp *h)
{
    const size_t M = h->members, Bp = h->Bp_max;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t s_par = al(M * kPS * sizeof(float));
    const size_t s_w = al(M * kPS * sizeof(uint16_t));
    const size_t s_wt = al(M * kTS * sizeof(uint16_t));
    const size_t s_z = al(M * 3 * Bp * kH * sizeof(float));
    const size_t s_a0t = al(M * 32 * Bp * sizeof(uint16_t));
    const size_t s_at = al(M * 3 * kH * Bp * sizeof(uint16_t));
    const size_t s_d4t = al(M * 16 * Bp * sizeof(uint16_t));
    const size_t s_lp = al(M * (Bp / kTM) * sizeof(float));
    const size_t s_l = al(M * sizeof(float));
    const size_t total = 4 * s_par + s_w + s_wt + s_z + s_a0t + 2 * s_at + s_d4t + s_lp + s_l;
    if (hipMalloc(&h->block, total) != hipSuccess) return fail(VQD_E_NOMEM, "surrogate allocation failed");
    char *p = static_cast<char *>(h->block);
    auto take = [&](size_t s) { char *q = p; p += s; return q; };
    h->theta = reinterpret_cast<float *>(take(s_par));
    h->m1 = reinterpret_cast<float *>(take(s_par));
    h->m2 = reinterpret_cast<float *>(take(s_par));
    h->grad = reinterpret_cast<float *>(take(s_par));
    h->w = reinterpret_cast<uint16_t *>(take(s_w));
    h->wt = reinterpret_cast<uint16_t *>(take(s_wt));
    h->z = reinterpret_cast<float *>(take(s_z));
    h->a0t = reinterpret_cast<uint16_t *>(take(s_a0t));
    h->at = reinterpret_cast<uint16_t *>(take(s_at));
    h->dt = reinterpret_cast<uint16_t *>(take(s_at));
    h->d4t = reinterpret_cast<uint16_t *>(take(s_d4t));
    h->loss_part = reinterpret_cast<float *>(take(s_lp));
    h->loss = reinterpret_cast<float *>(take(s_l));
    VQD_HIP(hipMemset(h->block, 0, total));
    return VQD_OK;
}

int check_mlp(const vqd_mlp *h)
{
    if (!h) return fail(VQD_E_ARG, "null surrogate");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
        return fail(VQD_E_ARG, "surrogate used on another device than it was created on");
    return VQD_OK;
}

int refresh_copies(vqd_mlp *h, hipStream_t st, bool apply, float lr)
{
    AdamArgs a{};
    a.members = h->members;
    a.apply = apply ? 1 : 0;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.omb1 = (float)(1.0 - 0.9);
    a.omb2 = (float)(1.0 - 0.999);
    a.eps = 1e-8f;
    if (apply) {
        a.c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)h->step)));
        a.c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)h->step)));
    }
    a.theta = h->theta;
    a.m1 = h->m1;
    a.m2 = h->m2;
    a.grad = h->grad;
    a.w = h->w;
    a.wt = h->wt;
    hipLaunchKernelGGL(k_mlp_adam, dim3(1024), dim3(256), 0, st, a);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int run_grad(vqd_mlp *h, const float *x, const float *y, const int *idx, int B, hipStream_t st)
{
    if (!x || !y) return fail(VQD_E_ARG, "null input");
    if (B < 1 || B > h->max_batch) return fail(VQD_E_SIZE, "batch size out of range");
    const int Bp = (B + kTM - 1) / kTM * kTM;
    FwdArgs f{};
    f.x = x;
    f.idx = idx;
    f.y = y;
    f.B = B;
    f.Bp = Bp;
    f.members = h->members;
    f.grad_scale = 2.0f / ((float)B * (float)kOut);
    f.w = h->w;
    f.theta = h->theta;
    f.z = h->z;
    f.a0t = h->a0t;
    f.at = h->at;
    f.d4t = h->d4t;
    f.loss_part = h->loss_part;
    hipLaunchKernelGGL(k_mlp_fwd_train, dim3(Bp / kTM, h->members), dim3(256), 0, st, f);
    VQD_HIP(hipGetLastError());
    BwdArgs b{};
    b.Bp = Bp;
    b.wt = h->wt;
    b.z = h->z;
    b.d4t = h->d4t;
    b.dt = h->dt;
    hipLaunchKernelGGL(k_mlp_bwd, dim3(Bp / kTM, h->members), dim3(256), 0, st, b);
    VQD_HIP(hipGetLastError());
    WgradArgs g{};
    g.Bp = Bp;
    g.a0t = h->a0t;
    g.at = h->at;
    g.d4t = h->d4t;
    g.dt = h->dt;
    g.grad = h->grad;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(kWgradTiles, h->members), dim3(256), 0, st, g);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(64), 0, st, (const float *)h->loss_part, Bp / kTM, h->members,
                       1.0f / ((float)B * (float)kOut), h->loss);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

}  // namespace

extern "C" {

int vqd_mlp_create(int members, int max_batch, vqd_mlp **out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output");
    *out = nullptr;
    if (members < 1 || members > kMaxMembers) return fail(VQD_E_SIZE, "members must be in [1, 8]");
    if (max_batch < 1 || max_batch > (1 << 20)) return fail(VQD_E_SIZE, "max_batch must be in [1, 2^20]");
    vqd_mlp *h = new (std::nothrow) vqd_mlp;
    if (!h) return fail(VQD_E_NOMEM, "host allocation failed");
    h->members = members;
    h->max_batch = max_batch;
    h->Bp_max = (max_batch + kTM - 1) / kTM * kTM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(VQD_E_HIP, "no HIP device");
    }
    if (int rc = mlp_alloc(h)) {
        delete h;
        return rc;
    }
    *out = h;
    return VQD_OK;
}

int vqd_mlp_destroy(vqd_mlp *h)
{
    clear_error();
    if (!h) return VQD_OK;
    if (h->block) {
        (void)hipDeviceSynchronize();
        (void)hipFree(h->block);
    }
    delete h;
    return VQD_OK;
}

int vqd_mlp_n_params(void) { return kP; }

int vqd_mlp_set_state(vqd_mlp *h, int which, const float *host)
{
    clear_error();
    if (int rc = check_mlp(h)) return rc;
    if (!host || which < VQD_MLP_PARAMS || which > VQD_MLP_ADAM_V) return fail(VQD_E_ARG, "bad state arguments");
    float *dst = which == VQD_MLP_PARAMS ? h->theta : which == VQD_MLP_ADAM_M ? h->m1 : h->m2;
    for (int m = 0; m < h->members; ++m) {
        for (int p = 0; p < kP; ++p)
            if (!std::isfinite(host[(size_t)m * kP + p])) return fail(VQD_E_ARG, "non-finite state value");
    }
    VQD_HIP(hipMemcpy2D(dst, kPS * sizeof(float), host, kP * sizeof(float), kP * sizeof(float), h->members,
                        hipMemcpyHostToDevice));
    if (which == VQD_MLP_PARAMS) {
        if (int rc = refresh_copies(h, nullptr, false, 0.f)) return rc;
        VQD_HIP(hipDeviceSynchronize());
    }
    return VQD_OK;
}

int vqd_mlp_get_state(const vqd_mlp *h, int which, float *host)
{
    clear_error();
    if (int rc = check_mlp(h)) return rc;
    if (!host || which < VQD_MLP_PARAMS || which > VQD_MLP_GRAD) return fail(VQD_E_ARG, "bad state arguments");
    const float *src = which == VQD_MLP_PARAMS ? h->theta : which == VQD_MLP_ADAM_M ? h->m1
                     : which == VQD_MLP_ADAM_V ? h->m2 : h->grad;
    VQD_HIP(hipDeviceSynchronize());
    VQD_HIP(hipMemcpy2D(host, kP * sizeof(float), src, kPS * sizeof(float), kP * sizeof(float), h->members,
                        hipMemcpyDeviceToHost));
    return VQD_OK;
}

int vqd_mlp_set_step(vqd_mlp *h, long long step)
{
    clear_error();
    if (!h || step < 0) return fail(VQD_E_ARG, "bad step");
    h->step = step;
    return VQD_OK;
}

long long vqd_mlp_get_step(const vqd_mlp *h) { return h ? h->step : -1; }

int vqd_mlp_grad(vqd_mlp *h, const float *x, const float *y, const int *idx, int B, float *loss_out,
                 void *hip_stream)
{
    clear_error();
    if (int rc = check_mlp(h)) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (int rc = run_grad(h, x, y, idx, B, st)) return rc;
    if (loss_out)
        VQD_HIP(hipMemcpyAsync(loss_out, h->loss, h->members * sizeof(float), hipMemcpyDeviceToDevice, st));
    return VQD_OK;
}

int vqd_mlp_train_step(vqd_mlp *h, const float *x, const float *y, const int *idx, int B, float lr,
                       float *loss_out, void *hip_stream)
{
    clear_error();
    if (int rc = check_mlp(h)) return rc;
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(VQD_E_ARG, "bad learning rate");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (int rc = run_grad(h, x, y, idx, B, st)) return rc;
    h->step += 1;
    if (int rc = refresh_copies(h, st, true, lr)) return rc;
    if (loss_out)
        VQD_HIP(hipMemcpyAsync(loss_out, h->loss, h->members * sizeof(float), hipMemcpyDeviceToDevice, st));
    return VQD_OK;
}

int vqd_mlp_predict(const vqd_mlp *h, const float *x, int B, float *mean, float *spread, float *member_out,
                    void *hip_stream)
{
    clear_error();
    if (int rc = check_mlp(h)) return rc;
    if (!x || !mean || !spread) return fail(VQD_E_ARG, "null argument");
    if (B < 0) return fail(VQD_E_SIZE, "negative batch");
    if (B == 0) return VQD_OK;
    FwdArgs f{};
    f.x = x;
    f.B = B;
    f.members = h->members;
    f.w = h->w;
    f.theta = h->theta;
    f.mean = mean;
    f.spread = spread;
    f.member_out = member_out;
    const unsigned blocks = (unsigned)((B + kTM - 1) / kTM);
    hipLaunchKernelGGL(k_mlp_predict, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(hip_stream), f);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

}  // extern "C"
