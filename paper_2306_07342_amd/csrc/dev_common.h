// Device helpers shared by the gfx950 kernels of the vqd library: bit
// deposit, LDS swizzle, uniform values, coefficient access and the dense
// small-matrix application on the 16 register slots of a thread.
#pragma once

#include <hip/hip_runtime.h>

#include "vqd_internal.h"

namespace vqd {
namespace {

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

// LDS index swizzle (see lds_swizzle).
__device__ __forceinline__ uint32_t swz(uint32_t l) { return lds_swizzle(l); }

__device__ __forceinline__ uint32_t uni(uint32_t x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

// Coefficient c of an op: complex entries as stored, real ones packed two
// per pool entry.
template <bool REAL>
__device__ __forceinline__ double2 coef(const double2 *__restrict__ M, int c)
{
    if (REAL) {
        const double2 p = M[c >> 1];
        return make_double2((c & 1) ? p.y : p.x, 0.0);
    }
    return M[c];
}

template <bool REAL>
__device__ __forceinline__ void cmac(double2 &y, const double2 m, const double2 x)
{
    y.x = fma(m.x, x.x, y.x);
    y.y = fma(m.x, x.y, y.y);
    if (!REAL) {
        y.x = fma(-m.y, x.y, y.x);
        y.y = fma(m.y, x.x, y.y);
    }
}

// Dense matrix on the register bits in MASK (column-major coefficients), for
// every setting of the other register bits.  Column-outer order: each
// coefficient column feeds DIM * NG independent accumulators; the first
// column initialises them.
template <int MASK, bool REAL>
__device__ __forceinline__ void apply_mat(const double2 (&a)[16], double2 (&y)[16], const double2 *__restrict__ M)
{
    constexpr int NB = popc4(MASK), DIM = 1 << NB, NG = 16 >> NB, REST = (~MASK) & 15;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        double2 col[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) col[i] = coef<REAL>(M, j * DIM + i);
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int so = dep4(i, MASK) | dep4(g, REST), si = dep4(j, MASK) | dep4(g, REST);
                if (j == 0) {
                    y[so].x = col[i].x * a[si].x;
                    y[so].y = col[i].x * a[si].y;
                    if (!REAL) {
                        y[so].x = fma(-col[i].y, a[si].y, y[so].x);
                        y[so].y = fma(col[i].y, a[si].x, y[so].y);
                    }
                } else {
                    cmac<REAL>(y[so], col[i], a[si]);
                }
            }
    }
}

// KOP_PTM on the register bits in MASK (the row and column bit of one
// qubit): per group of 4 slots, the block B (B[u][v] at local index u + 2v)
// has Pauli components a_I = B00 + B11, a_Z = B00 - B11, a_X = B01 + B10,
// a_Y = i (B01 - B10); the map keeps a_I, h = (R / 2) a for the rows X, Y,
// Z of its real transfer matrix R, and the new block is B00 = a_I / 2 + h_Z,
// B11 = a_I / 2 - h_Z, B01 = h_X - i h_Y, B10 = h_X + i h_Y.  Group by group;
// the scheduling barrier between groups keeps the compiler from
// interleaving them, which would hold every group's temporaries at once.
template <int MASK>
__device__ __forceinline__ void apply_ptm(const double2 (&x)[16], double2 (&y)[16], const double2 *__restrict__ M)
{
    constexpr int REST = (~MASK) & 15;
    double c[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = coef<true>(M, k).x;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int s0 = dep4(0, MASK) | dep4(g, REST), s1 = dep4(1, MASK) | dep4(g, REST);
        const int s2 = dep4(2, MASK) | dep4(g, REST), s3 = dep4(3, MASK) | dep4(g, REST);
        const double2 aI = make_double2(x[s0].x + x[s3].x, x[s0].y + x[s3].y);
        const double2 aX = make_double2(x[s2].x + x[s1].x, x[s2].y + x[s1].y);
        const double2 d = make_double2(x[s2].x - x[s1].x, x[s2].y - x[s1].y);     // a_Y = i d
        const double2 aZ = make_double2(x[s0].x - x[s3].x, x[s0].y - x[s3].y);
        double2 h[3];      // X, Y, Z
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double *w = c + 4 * r;   // columns I, X, Y, Z
            h[r].x = fma(w[3], aZ.x, fma(-w[2], d.y, fma(w[1], aX.x, w[0] * aI.x)));
            h[r].y = fma(w[3], aZ.y, fma(w[2], d.x, fma(w[1], aX.y, w[0] * aI.y)));
        }
        y[s0] = make_double2(fma(0.5, aI.x, h[2].x), fma(0.5, aI.y, h[2].y));
        y[s3] = make_double2(fma(0.5, aI.x, -h[2].x), fma(0.5, aI.y, -h[2].y));
        y[s2] = make_double2(h[0].x + h[1].y, h[0].y - h[1].x);
        y[s1] = make_double2(h[0].x - h[1].y, h[0].y + h[1].x);
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ double2 cmul(const double2 m, const double2 x)
{
    return make_double2(fma(m.x, x.x, -m.y * x.y), fma(m.x, x.y, m.y * x.x));
}

// Local index bits of register slot e (rl[b] = local bit of register bit b).
__device__ __forceinline__ uint32_t slot_l(const uint32_t (&rl)[4], int e)
{
    return ((e & 1) ? rl[0] : 0) | ((e & 2) ? rl[1] : 0) | ((e & 4) ? rl[2] : 0) | ((e & 8) ? rl[3] : 0);
}

// Thread id of this lane within the workgroup, from the wave's base (the
// lane count is opaque to the compiler, so values derived from it are
// recomputed rather than kept live).
__device__ __forceinline__ uint32_t lane_tid(uint32_t wave_base)
{
    return wave_base + __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

}  // namespace
}  // namespace vqd
