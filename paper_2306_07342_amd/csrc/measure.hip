// gfx950 kernels of measurement on the density matrix.
//
// * k_project    -- collapse after a projective measurement: every element
//                   rho[r][c] whose row r or column c lies outside the
//                   measured projector's support becomes zero, the others are
//                   divided by the outcome's weight.  Zeroed elements are
//                   written without being read.
// * k_diag_probs -- the diagonal probabilities max(0, Re rho[x][x]) into a
//                   contiguous array.
// * k_cdf        -- their running sums in one workgroup: per-thread runs
//                   of consecutive terms, chained by thread totals
//                   (2^n <= 65536 terms).
// * k_sample     -- one basis state per uniform: binary search of the
//                   running sums for the first one above u W.
#include <hip/hip_runtime.h>

#include "vqd_internal.h"

namespace vqd {

namespace {

constexpr int kMeasThreads = 256;

// Support of the projector: bit q0 equal to m (kind MEAS_Z), or the parity of
// bits q0 and q1 odd for m = 0 and even for m = 1 (kind MEAS_PARITY).
__device__ __forceinline__ bool in_support(uint64_t x, uint32_t kind, uint32_t q0, uint32_t q1, uint32_t m)
{
    if (kind == MEAS_Z) return ((x >> q0) & 1u) == m;
    const uint32_t par = (uint32_t)(((x >> q0) ^ (x >> q1)) & 1u);
    return par == (m ^ 1u);
}

__global__ void __launch_bounds__(kMeasThreads)
k_project(double2 *__restrict__ amps, uint32_t n, uint32_t kind, uint32_t q0, uint32_t q1, uint32_t m,
          double scale)
{
    const uint64_t total = 1ull << (2 * n), mask = (1ull << n) - 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const bool keep = in_support(i & mask, kind, q0, q1, m) && in_support(i >> n, kind, q0, q1, m);
        double2 v = make_double2(0.0, 0.0);
        if (keep) {
            v = amps[i];
            v.x *= scale;
            v.y *= scale;
        }
        amps[i] = v;
    }
}

__global__ void __launch_bounds__(kMeasThreads)
k_diag_probs(const double2 *__restrict__ amps, uint32_t n, double *__restrict__ p)
{
    const uint64_t D = 1ull << n;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < D; x += (uint64_t)gridDim.x * blockDim.x)
        p[x] = fmax(0.0, amps[x + (x << n)].x);
}

// cum[x] = p[0] + ... + p[x]; cum[D] holds the last x with p[x] > 0 (or 0),
// as a double.  One workgroup: thread t owns the C = D / 256 consecutive
// terms from t C (all D when D < 256, in thread 0) and forms their running
// sums l_j left to right; thread 0 chains the thread totals,
// P_(t+1) = P_t + l_last(t); then cum[t C + j] = P_t + l_j.  Each sum is
// rounded once onto P_t and P_(t+1) is the same rounding of thread t's last
// sum, so the sums never decrease across thread boundaries either (the
// binary search of k_sample relies on it).  They differ from a single
// left-to-right chain only in rounding.
constexpr int kCdfThreads = 256;

__global__ void __launch_bounds__(kCdfThreads) k_cdf(const double *__restrict__ p, uint32_t n, double *__restrict__ cum)
{
    __shared__ double pre[kCdfThreads + 1];
    __shared__ int lastpos[kCdfThreads];
    const uint32_t t = threadIdx.x, D = 1u << n;
    const uint32_t C = (D >= (uint32_t)kCdfThreads) ? D / kCdfThreads : D;
    const uint32_t T = D / C;                   // threads with terms
    const uint32_t x0 = t * C;
    double l = 0.0;
    int lp = -1;
    if (t < T) {
        for (uint32_t j = 0; j < C; ++j) {
            const double v = p[x0 + j];
            l += v;
            lp = (v > 0.0) ? (int)(x0 + j) : lp;
        }
    }
    pre[t + 1] = l;
    lastpos[t] = lp;
    __syncthreads();
    if (t == 0) {
        double P = 0.0;
        int last = 0;
        for (uint32_t k = 0; k < T; ++k) {
            const double tot = pre[k + 1];
            pre[k] = P;                             // thread k's offset
            P += tot;
            last = (lastpos[k] >= 0) ? lastpos[k] : last;
        }
        cum[D] = (double)last;
    }
    __syncthreads();
    if (t < T) {
        const double P = pre[t];
        l = 0.0;
        for (uint32_t j = 0; j < C; ++j) {
            l += p[x0 + j];
            cum[x0 + j] = P + l;
        }
    }
}

__global__ void __launch_bounds__(kMeasThreads)
k_sample(const double *__restrict__ cum, uint32_t n, const double *__restrict__ U, uint64_t shots,
         uint32_t *__restrict__ out)
{
    const uint32_t D = 1u << n;
    const double W = cum[D - 1];
    const uint32_t last = (uint32_t)cum[D];
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < shots;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const double thr = U[s] * W;
        // first x with cum[x] > thr (the sums never decrease)
        uint32_t lo = 0, hi = D;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (cum[mid] > thr) hi = mid;
            else lo = mid + 1;
        }
        out[s] = (lo < D) ? lo : last;
    }
}

uint32_t grid_for(uint64_t work)
{
    uint64_t blocks = (work + kMeasThreads - 1) / kMeasThreads;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    return (uint32_t)blocks;
}

}  // namespace

int launch_project(double2 *amps, int n, int kind, int q0, int q1, int m, double scale, hipStream_t st)
{
    hipLaunchKernelGGL(k_project, dim3(grid_for(1ull << (2 * n))), dim3(kMeasThreads), 0, st, amps, (uint32_t)n,
                       (uint32_t)kind, (uint32_t)q0, (uint32_t)q1, (uint32_t)m, scale);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int launch_sample(const double2 *amps, int n, double *scratch, const double *U, uint64_t shots, uint32_t *out,
                  hipStream_t st)
{
    const uint64_t D = 1ull << n;
    double *p = scratch, *cum = scratch + D;
    hipLaunchKernelGGL(k_diag_probs, dim3(grid_for(D)), dim3(kMeasThreads), 0, st, amps, (uint32_t)n, p);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cdf, dim3(1), dim3(kCdfThreads), 0, st, p, (uint32_t)n, cum);
    VQD_HIP(hipGetLastError());
    if (shots == 0) return VQD_OK;
    hipLaunchKernelGGL(k_sample, dim3(grid_for(shots)), dim3(kMeasThreads), 0, st, cum, (uint32_t)n, U, shots, out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

}  // namespace vqd
