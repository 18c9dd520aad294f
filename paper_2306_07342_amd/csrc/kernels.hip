// gfx950 kernels of the vqd library.
//
// * k_pass     -- one HBM pass over the vectorised density matrix applying a
//                 planned sequence of register phases (see vqd_internal.h).
// * k_init     -- |b><b| and the product-diagonal (thermal) initial states.
// * k_purity / k_diag / k_zz / k_pauli -- read-out reductions (wave shuffles,
//                 then one partial per workgroup, then a fixed-order second
//                 stage, so results are deterministic).
#include <hip/hip_runtime.h>

#include "vqd_internal.h"

namespace vqd {

namespace {

constexpr int kThreads = 256;

// Deposit the low bits of v into the set bits of mask (ascending order).
__host__ __device__ constexpr int dep4(int v, int mask)
{
    int out = 0, k = 0;
    for (int b = 0; b < 4; ++b)
        if (mask >> b & 1) {
            if (v >> k & 1) out |= 1 << b;
            ++k;
        }
    return out;
}

__host__ __device__ constexpr int popc4(int m)
{
    return (m & 1) + (m >> 1 & 1) + (m >> 2 & 1) + (m >> 3 & 1);
}

// LDS index swizzle: xor the low 3 bits of the local index with a hash of
// the higher bits so that strided register phases spread over the banks.
__device__ __forceinline__ uint32_t swz(uint32_t l)
{
    return l ^ (((l >> 3) ^ (l >> 6) ^ (l >> 9)) & 7u);
}

__device__ __forceinline__ uint32_t uni(uint32_t x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

// y <- M x on the register bits in MASK, for every setting of the other bits.
template <int MASK>
__device__ __forceinline__ void apply_mat(double2 (&a)[16], const KOp *__restrict__ op,
                                          const double2 *__restrict__ M)
{
    constexpr int NB = popc4(MASK);
    constexpr int DIM = 1 << NB;
    constexpr int NG = 16 >> NB;
    constexpr int REST = (~MASK) & 15;
    uint32_t nz[(DIM * DIM + 31) / 32], cx[(DIM * DIM + 31) / 32];
#pragma unroll
    for (int w = 0; w < (DIM * DIM + 31) / 32; ++w) {
        nz[w] = uni(op->nz[w]);
        cx[w] = uni(op->cx[w]);
    }
    double2 y[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) y[e] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            const int bit = i * DIM + j;
            if ((nz[bit >> 5] >> (bit & 31)) & 1u) {
                const double2 m = M[bit];
                if ((cx[bit >> 5] >> (bit & 31)) & 1u) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const int so = dep4(i, MASK) | dep4(g, REST);
                        const int si = dep4(j, MASK) | dep4(g, REST);
                        y[so].x = fma(m.x, a[si].x, y[so].x);
                        y[so].y = fma(m.x, a[si].y, y[so].y);
                        y[so].x = fma(-m.y, a[si].y, y[so].x);
                        y[so].y = fma(m.y, a[si].x, y[so].y);
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const int so = dep4(i, MASK) | dep4(g, REST);
                        const int si = dep4(j, MASK) | dep4(g, REST);
                        y[so].x = fma(m.x, a[si].x, y[so].x);
                        y[so].y = fma(m.x, a[si].y, y[so].y);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) a[e] = y[e];
}

// Element-wise factors indexed by the slot (register bits).
__device__ __forceinline__ void apply_diag(double2 (&a)[16], const KOp *__restrict__ op,
                                           const double2 *__restrict__ M)
{
    const uint32_t nz = uni(op->nz[0]), cx = uni(op->cx[0]);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if ((nz >> e) & 1u) {
            const double2 m = M[e];
            if ((cx >> e) & 1u) {
                const double re = a[e].x * m.x - a[e].y * m.y;
                const double im = a[e].x * m.y + a[e].y * m.x;
                a[e] = make_double2(re, im);
            } else {
                a[e].x *= m.x;
                a[e].y *= m.x;
            }
        }
    }
}

__device__ __forceinline__ uint32_t gather_bits(uint64_t gi, const uint32_t (&pos)[4], uint32_t nb)
{
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if ((uint32_t)j < nb) r |= (uint32_t)((gi >> pos[j]) & 1u) << j;
    return r;
}

// Element-wise factors indexed by arbitrary global bits.
__device__ __forceinline__ void apply_diag_rt(double2 (&a)[16], const KOp *__restrict__ op,
                                              const double2 *__restrict__ M, uint64_t base,
                                              const uint64_t (&rg)[4])
{
    const uint32_t nb = uni(op->nbits);
    uint32_t pos[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) pos[j] = uni(op->gpos[j]);
    const uint32_t rt = gather_bits(base, pos, nb);
    if (!uni(op->regdep)) {
        const double2 m = M[rt];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const double re = a[e].x * m.x - a[e].y * m.y;
            const double im = a[e].x * m.y + a[e].y * m.x;
            a[e] = make_double2(re, im);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint64_t ge = ((e & 1) ? rg[0] : 0) | ((e & 2) ? rg[1] : 0) |
                                ((e & 4) ? rg[2] : 0) | ((e & 8) ? rg[3] : 0);
            const uint32_t ct = gather_bits(ge, pos, nb);
            const double2 m = M[rt | ct];
            const double re = a[e].x * m.x - a[e].y * m.y;
            const double im = a[e].x * m.y + a[e].y * m.x;
            a[e] = make_double2(re, im);
        }
    }
}

__global__ void __launch_bounds__(kThreads)
k_pass(double2 *__restrict__ amps, const KPass *__restrict__ passes,
       const KPhase *__restrict__ phases, const KOp *__restrict__ ops,
       const double2 *__restrict__ mats, uint32_t pass_idx)
{
    extern __shared__ double2 lds[];
    const KPass *P = passes + pass_idx;
    const uint32_t L = uni(P->L);
    const uint32_t nthr = L - 4;
    uint64_t tile = blockIdx.x;
    if (uni(P->xcd_swizzle)) {
        // workgroup b runs on XCD b % 8: give consecutive workgroups of one
        // XCD the tiles that differ in the lowest group bits
        const uint64_t x = tile & 7u, s = tile >> 3;
        tile = (s & 7u) | (x << 3) | ((s >> 3) << 6);
    }
    uint64_t gbase = 0;
    const uint32_t ngb = uni(P->n_group_bits);
    for (uint32_t i = 0; i < ngb; ++i)
        gbase |= ((tile >> i) & 1ull) << uni(P->group_gpos[i]);

    const uint32_t tid = threadIdx.x;
    const uint32_t pb = uni(P->phase_begin), pe = uni(P->phase_end);
    const bool phantom = uni(P->phantom) != 0;
    double2 a[16];

    for (uint32_t ph = pb; ph < pe; ++ph) {
        const KPhase *H = phases + ph;
        uint32_t tl = 0;
        uint64_t tg = 0;
        for (uint32_t i = 0; i < nthr; ++i) {
            const uint32_t b = (tid >> i) & 1u;
            tl |= b << uni(H->thr_local[i]);
            tg |= (uint64_t)b << uni(H->thr_gpos[i]);
        }
        uint32_t rl[4];
        uint64_t rg[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            rl[b] = 1u << uni(H->reg_local[b]);
            rg[b] = 1ull << uni(H->reg_gpos[b]);
        }
        const uint64_t base = gbase | tg;
        if (ph == pb) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint64_t gi = base | ((e & 1) ? rg[0] : 0) | ((e & 2) ? rg[1] : 0) |
                                    ((e & 4) ? rg[2] : 0) | ((e & 8) ? rg[3] : 0);
                if (phantom && (gi >> kPhantomPos))
                    a[e] = make_double2(0.0, 0.0);
                else
                    a[e] = amps[gi];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t li = tl | ((e & 1) ? rl[0] : 0) | ((e & 2) ? rl[1] : 0) |
                                    ((e & 4) ? rl[2] : 0) | ((e & 8) ? rl[3] : 0);
                a[e] = lds[swz(li)];
            }
            __syncthreads();
        }

        const uint32_t ob = uni(H->op_begin), oe = uni(H->op_end);
        for (uint32_t oi = ob; oi < oe; ++oi) {
            const KOp *op = ops + oi;
            const uint32_t kind = uni(op->kind);
            const double2 *M = mats + uni(op->mat);
            if (kind == KOP_MAT) {
                switch (uni(op->opmask)) {
                case 5: apply_mat<5>(a, op, M); break;
                case 10: apply_mat<10>(a, op, M); break;
                case 15: apply_mat<15>(a, op, M); break;
                case 7: apply_mat<7>(a, op, M); break;
                default: break;
                }
            } else if (kind == KOP_DIAG) {
                apply_diag(a, op, M);
            } else {
                apply_diag_rt(a, op, M, base, rg);
            }
        }

        if (ph + 1 < pe) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t li = tl | ((e & 1) ? rl[0] : 0) | ((e & 2) ? rl[1] : 0) |
                                    ((e & 4) ? rl[2] : 0) | ((e & 8) ? rl[3] : 0);
                lds[swz(li)] = a[e];
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint64_t gi = base | ((e & 1) ? rg[0] : 0) | ((e & 2) ? rg[1] : 0) |
                                    ((e & 4) ? rg[2] : 0) | ((e & 8) ? rg[3] : 0);
                if (!(phantom && (gi >> kPhantomPos))) amps[gi] = a[e];
            }
        }
    }
}

// ------------------------------------------------------------------ init --
struct InitArgs {
    double p0[VQD_MAX_QUBITS];
};

// mode 0: amp[target] = 1, all other amplitudes 0.
// mode 1: product-diagonal state from p0 (ground-state populations).
__global__ void __launch_bounds__(kThreads)
k_init(double2 *__restrict__ amps, uint64_t count, int n, int mode, uint64_t target, InitArgs args)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t D = 1ull << n, mask = D - 1;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        double v = 0.0;
        if (mode == 0) {
            v = (i == target) ? 1.0 : 0.0;
        } else {
            const uint64_t r = i & mask, c = i >> n;
            if (r == c) {
                v = 1.0;
                for (int j = 0; j < n; ++j) v *= ((r >> j) & 1u) ? (1.0 - args.p0[j]) : args.p0[j];
            }
        }
        amps[i] = make_double2(v, 0.0);
    }
}

// ------------------------------------------------------------ reductions --
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of NV values per thread over the block; thread 0 gets the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *smem /* NV * 4 */)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) smem[k * 4 + wv] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = (smem[k * 4] + smem[k * 4 + 1]) + (smem[k * 4 + 2] + smem[k * 4 + 3]);
    }
}

constexpr int kRedBlocks = 1024;

__global__ void __launch_bounds__(kThreads)
k_purity(const double2 *__restrict__ amps, uint64_t count, double *__restrict__ partials)
{
    __shared__ double smem[4];
    double acc[1] = {0.0};
    double acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < count; i += 4 * stride) {
        const double2 x0 = amps[i], x1 = amps[i + stride], x2 = amps[i + 2 * stride],
                      x3 = amps[i + 3 * stride];
        acc[0] = fma(x0.x, x0.x, fma(x0.y, x0.y, acc[0]));
        acc1 = fma(x1.x, x1.x, fma(x1.y, x1.y, acc1));
        acc2 = fma(x2.x, x2.x, fma(x2.y, x2.y, acc2));
        acc3 = fma(x3.x, x3.x, fma(x3.y, x3.y, acc3));
    }
    for (; i < count; i += stride) {
        const double2 x = amps[i];
        acc[0] = fma(x.x, x.x, fma(x.y, x.y, acc[0]));
    }
    acc[0] = (acc[0] + acc1) + (acc2 + acc3);
    block_sum<1>(acc, smem);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// Fixed-order sum of nb partials of NV values each (layout [block][value]).
__global__ void __launch_bounds__(kThreads)
k_finish(const double *__restrict__ partials, int nb, int nv, double *__restrict__ out)
{
    __shared__ double smem[4];
    for (int k = 0; k < nv; ++k) {
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nb; b += blockDim.x) v[0] += partials[(size_t)b * nv + k];
        block_sum<1>(v, smem);
        if (threadIdx.x == 0) out[k] = v[0];
        __syncthreads();
    }
}

// Diagonal read-out: trace (re, im), <Z_i> and optionally the probabilities.
// partials layout: [block][2 + n].
__global__ void __launch_bounds__(kThreads)
k_diag(const double2 *__restrict__ amps, int n, double *__restrict__ probs,
       double *__restrict__ partials)
{
    __shared__ double smem[(2 + VQD_MAX_QUBITS) * 4];
    double v[2 + VQD_MAX_QUBITS];
#pragma unroll
    for (int k = 0; k < 2 + VQD_MAX_QUBITS; ++k) v[k] = 0.0;
    const uint64_t D = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < D; r += stride) {
        const double2 x = amps[r * (D + 1)];
        if (probs) probs[r] = x.x;
        v[0] += x.x;
        v[1] += x.y;
#pragma unroll
        for (int q = 0; q < VQD_MAX_QUBITS; ++q)
            if (q < n) v[2 + q] += ((r >> q) & 1u) ? -x.x : x.x;
    }
    block_sum<2 + VQD_MAX_QUBITS>(v, smem);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 2 + VQD_MAX_QUBITS; ++k)
            if (k < 2 + n) partials[(size_t)blockIdx.x * (2 + n) + k] = v[k];
    }
}

// <Z_i Z_j>: one workgroup per pair over the contiguous probabilities.
__global__ void __launch_bounds__(kThreads)
k_zz(const double *__restrict__ probs, int n, const int2 *__restrict__ pairs,
     double *__restrict__ out)
{
    __shared__ double smem[4];
    const int2 pr = pairs[blockIdx.x];
    const uint64_t D = 1ull << n;
    double v[1] = {0.0};
    for (uint64_t r = threadIdx.x; r < D; r += blockDim.x) {
        const double p = probs[r];
        v[0] += (((r >> pr.x) ^ (r >> pr.y)) & 1u) ? -p : p;
    }
    block_sum<1>(v, smem);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// Tr(P rho) = sum_r phi(r) rho[r][r ^ x], phi(r) = i^{ny} (-1)^{|r & zmask|}.
__global__ void __launch_bounds__(kThreads)
k_pauli(const double2 *__restrict__ amps, int n, uint64_t xmask, uint64_t zmask,
        double *__restrict__ partials)
{
    __shared__ double smem[8];
    double v[2] = {0.0, 0.0};
    const uint64_t D = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < D; r += stride) {
        const double2 x = amps[r + D * (r ^ xmask)];
        const bool neg = __popcll(r & zmask) & 1;
        v[0] += neg ? -x.x : x.x;
        v[1] += neg ? -x.y : x.y;
    }
    block_sum<2>(v, smem);
    if (threadIdx.x == 0) {
        partials[(size_t)blockIdx.x * 2] = v[0];
        partials[(size_t)blockIdx.x * 2 + 1] = v[1];
    }
}

}  // namespace

// ------------------------------------------------------------- launches --
int launch_pass(double2 *amps, const DevProgram &dev, const KPass &pass, uint32_t pass_idx,
                hipStream_t stream)
{
    const uint32_t threads = 1u << (pass.L - 4);
    const size_t lds = (pass.phase_end - pass.phase_begin > 1) ? (size_t(16) << pass.L) : 0;
    if (pass.n_tiles > 0xffffffffull) return fail(VQD_E_SIZE, "too many tiles for one launch");
    static bool attr_set = false;
    if (!attr_set) {
        VQD_HIP(hipFuncSetAttribute((const void *)k_pass, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    16 << kMaxTileBits));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_pass, dim3((uint32_t)pass.n_tiles), dim3(threads), lds, stream, amps,
                       dev.passes, dev.phases, dev.ops, dev.mats, pass_idx);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int launch_init(double2 *amps, int n, int mode, uint64_t b, const double *p0, hipStream_t stream)
{
    InitArgs args{};
    if (p0)
        for (int j = 0; j < n; ++j) args.p0[j] = p0[j];
    const uint64_t count = 1ull << (2 * n);
    uint64_t blocks = (count + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_init, dim3((uint32_t)blocks), dim3(kThreads), 0, stream, amps, count, n,
                       mode, b, args);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int ensure_scratch(ReduceScratch &s, size_t dev_doubles, size_t host_doubles)
{
    if (s.cap < dev_doubles) {
        if (s.dev) (void)hipFree(s.dev);
        s.dev = nullptr;
        s.cap = 0;
        if (hipMalloc(&s.dev, dev_doubles * sizeof(double)) != hipSuccess)
            return fail(VQD_E_NOMEM, "reduction scratch allocation failed");
        s.cap = dev_doubles;
    }
    if (s.host_cap < host_doubles) {
        if (s.host) (void)hipHostFree(s.host);
        s.host = nullptr;
        s.host_cap = 0;
        if (hipHostMalloc(&s.host, host_doubles * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(VQD_E_NOMEM, "pinned staging allocation failed");
        s.host_cap = host_doubles;
    }
    return VQD_OK;
}

void free_scratch(ReduceScratch &s)
{
    if (s.dev) (void)hipFree(s.dev);
    if (s.host) (void)hipHostFree(s.host);
    s = ReduceScratch{};
}

int reduce_purity(const double2 *amps, int n, ReduceScratch &s, hipStream_t st, double *out)
{
    int rc = ensure_scratch(s, kRedBlocks + 8, 8);
    if (rc) return rc;
    const uint64_t count = 1ull << (2 * n);
    uint64_t blocks = (count + kThreads - 1) / kThreads;
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL(k_purity, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, count, s.dev);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, s.dev, (int)blocks, 1, s.dev + kRedBlocks);
    VQD_HIP(hipGetLastError());
    VQD_HIP(hipMemcpyAsync(s.host, s.dev + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
    VQD_HIP(hipStreamSynchronize(st));
    *out = s.host[0];
    return VQD_OK;
}

int reduce_diag(const double2 *amps, int n, ReduceScratch &s, hipStream_t st, double *trace2,
                double *z, double *probs)
{
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    const size_t nv = 2 + n;
    const size_t off_res = blocks * nv, off_probs = off_res + nv;
    int rc = ensure_scratch(s, off_probs + (probs ? D : 0), nv + (probs ? D : 0));
    if (rc) return rc;
    hipLaunchKernelGGL(k_diag, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n,
                       probs ? s.dev + off_probs : nullptr, s.dev);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, s.dev, (int)blocks, (int)nv, s.dev + off_res);
    VQD_HIP(hipGetLastError());
    VQD_HIP(hipMemcpyAsync(s.host, s.dev + off_res, (nv + (probs ? D : 0)) * sizeof(double),
                           hipMemcpyDeviceToHost, st));
    VQD_HIP(hipStreamSynchronize(st));
    if (trace2) { trace2[0] = s.host[0]; trace2[1] = s.host[1]; }
    if (z) for (int q = 0; q < n; ++q) z[q] = s.host[2 + q];
    if (probs) for (uint64_t r = 0; r < D; ++r) probs[r] = s.host[nv + r];
    return VQD_OK;
}

int reduce_zz(const double2 *amps, int n, const int *pairs, int npairs, ReduceScratch &s,
              hipStream_t st, double *out)
{
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    const size_t nv = 2 + n;
    // layout: partials | probs | pairs (as int2 in doubles) | results
    const size_t off_probs = blocks * nv + nv;
    const size_t off_pairs = off_probs + D;
    const size_t off_out = off_pairs + npairs;
    int rc = ensure_scratch(s, off_out + npairs, (size_t)npairs * 2);
    if (rc) return rc;
    hipLaunchKernelGGL(k_diag, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n,
                       s.dev + off_probs, s.dev);
    VQD_HIP(hipGetLastError());
    int *hp = reinterpret_cast<int *>(s.host);
    for (int i = 0; i < 2 * npairs; ++i) hp[i] = pairs[i];
    VQD_HIP(hipMemcpyAsync(s.dev + off_pairs, hp, sizeof(int) * 2 * npairs, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_zz, dim3(npairs), dim3(kThreads), 0, st, s.dev + off_probs, n,
                       reinterpret_cast<const int2 *>(s.dev + off_pairs), s.dev + off_out);
    VQD_HIP(hipGetLastError());
    VQD_HIP(hipMemcpyAsync(s.host, s.dev + off_out, sizeof(double) * npairs, hipMemcpyDeviceToHost, st));
    VQD_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < npairs; ++i) out[i] = s.host[i];
    return VQD_OK;
}

int reduce_pauli(const double2 *amps, int n, uint64_t xmask, uint64_t zmask, int ny,
                 ReduceScratch &s, hipStream_t st, double *re, double *im)
{
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    int rc = ensure_scratch(s, blocks * 2 + 2, 2);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pauli, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n, xmask, zmask, s.dev);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, s.dev, (int)blocks, 2, s.dev + blocks * 2);
    VQD_HIP(hipGetLastError());
    VQD_HIP(hipMemcpyAsync(s.host, s.dev + blocks * 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    VQD_HIP(hipStreamSynchronize(st));
    // multiply by i^ny
    double a = s.host[0], b = s.host[1];
    for (int k = 0; k < (ny & 3); ++k) {
        const double t = a;
        a = -b;
        b = t;
    }
    *re = a;
    *im = b;
    return VQD_OK;
}

}  // namespace vqd
