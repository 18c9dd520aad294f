// gfx950 kernels of the Monte Carlo trajectory mode (state-vector samples,
// one Kraus operator drawn per channel; the paper's Sec. 2 alternative to the
// density matrix).
//
// * k_traj       -- a batch of trajectories.  A trajectory of n_eff qubits is
//                   held by 2^(n_eff-4) threads, 16 register slots each, and
//                   never leaves the chip: it starts as |0...0> in registers,
//                   every phase applies its ops to the register slots and
//                   moves the state through LDS to the next phase's layout,
//                   and only <Z_q>, the squared norm and (optionally) the
//                   final state are written to memory.  A channel's operator
//                   is drawn from the trajectory's uniform variate; for a
//                   general channel the weights ||K_i psi||^2 = Tr(K_i^dagger
//                   K_i rho_T) come from the reduced density matrix rho_T of
//                   the target qubits, summed over the trajectory's threads.
// * k_traj_stats -- mean and standard error over trajectories.
//
// Every sum over threads has a fixed order, so results are deterministic and
// all threads of a trajectory draw the same operator.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dev_common.h"
#include "vqd_internal.h"

namespace vqd {

namespace {

constexpr int kTrajRed = 16;          // values in one group reduction
constexpr int kTrajMaxWaves = 8;      // waves of the largest workgroup (512 threads)

__device__ __forceinline__ bool is_channel(uint32_t kind) { return kind == TOP_MIX || kind == TOP_KRAUS; }

struct TCtx {
    uint32_t tl;      // amplitude-index bits from the thread id
    uint32_t rl[4];   // amplitude-index bit of register bit b
};

// Amplitude-index bits of thread tt of a trajectory in phase H (thread bit i
// carries qubit thr_q[i]; unused entries are zero and tt has no bit there).
// The empty asm hides tt's value from the compiler, so the per-bit values are
// recomputed in every phase instead of being hoisted out of the phase loop
// and kept live (or spilled) across it.
__device__ __forceinline__ uint32_t traj_thread_bits(const TPhase *__restrict__ H, uint32_t tt)
{
    asm volatile("" : "+v"(tt));
    uint32_t tl = 0;
#pragma unroll
    for (uint32_t i = 0; i < (uint32_t)kTrajMaxThreadBits; ++i) tl |= ((tt >> i) & 1u) << (uni(H->thr_q[i]) & 31u);
    return tl;
}

// Sum of v over the threads of one trajectory, bitwise identical in all of
// them: inside the wave a butterfly (each pairwise sum is formed from the
// same two operands on both lanes; DPP steps for whole waves, lane shuffles
// below), then, when a trajectory spans several waves, the per-wave sums
// added in wave order through LDS.
// The cross-wave sums alternate between two LDS buffers (`flip`), so one
// barrier per reduction suffices: a buffer is written again only after every
// wave has passed the barrier of the reduction in between, which follows its
// reads of that buffer.
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_value(double x, int lane)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave, the same bits in every lane: lanes
// exchange with a partner in DPP steps (quad swaps, then mirror images
// within 8 and 16 lanes), each pair forming the same sum of the same two
// values, until each row of 16 holds its total; the four row totals are
// then added in a fixed order from scalar reads.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_partner<0xB1>(x);      // quad_perm [1, 0, 3, 2]
    x += dpp_partner<0x4E>(x);      // quad_perm [2, 3, 0, 1]
    x += dpp_partner<0x141>(x);     // row_half_mirror
    x += dpp_partner<0x140>(x);     // row_mirror
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

template <int CNT, bool WIDE>
__device__ __forceinline__ void group_sum(double (&v)[CNT], uint32_t log_tt, double *red, uint32_t wave,
                                          uint32_t wpt, uint32_t &flip)
{
    if (WIDE) {
#pragma unroll
        for (int i = 0; i < CNT; ++i) v[i] = wave_sum(v[i]);
    } else {
        for (uint32_t s = 0; s < log_tt; ++s) {
#pragma unroll
            for (int i = 0; i < CNT; ++i) v[i] += __shfl_xor(v[i], 1 << s);
        }
    }
    if (WIDE && wpt > 1) {
        double *buf = red + flip * (kTrajMaxWaves * kTrajRed);
        flip ^= 1u;
        if ((threadIdx.x & 63u) == 0) {
#pragma unroll
            for (int i = 0; i < CNT; ++i) buf[wave * kTrajRed + i] = v[i];
        }
        __syncthreads();
        // the trajectory's first wave and the wave count are wave-uniform
        const double *p = buf + uni((wave & ~(wpt - 1u)) * kTrajRed);
#pragma unroll
        for (int i = 0; i < CNT; ++i) v[i] = p[i];
        for (uint32_t w = 1; w < wpt; ++w) {
            p += kTrajRed;
#pragma unroll
            for (int i = 0; i < CNT; ++i) v[i] += p[i];
        }
    }
}

// This thread's part of the reduced density matrix of the register bits in
// MASK: rho_xy = sum over the other bits of psi_x conj(psi_y).  Packed as the
// DIM real diagonal entries, then (re, im) of rho_xy for x < y in row order.
template <int MASK>
__device__ __forceinline__ void rho_partial(const double2 (&a)[16], double (&r)[1 << (2 * popc4(MASK))])
{
    constexpr int NB = popc4(MASK), DIM = 1 << NB, NG = 16 >> NB, REST = (~MASK) & 15;
#pragma unroll
    for (int i = 0; i < DIM * DIM; ++i) r[i] = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        int p = 0;
#pragma unroll
        for (int x = 0; x < DIM; ++x) {
            const double2 ax = a[dep4(x, MASK) | dep4(g, REST)];
            r[x] = fma(ax.x, ax.x, fma(ax.y, ax.y, r[x]));
#pragma unroll
            for (int y = x + 1; y < DIM; ++y, ++p) {
                const double2 ay = a[dep4(y, MASK) | dep4(g, REST)];
                r[DIM + 2 * p] = fma(ax.x, ay.x, fma(ax.y, ay.y, r[DIM + 2 * p]));
                r[DIM + 2 * p + 1] = fma(ax.y, ay.x, fma(-ax.x, ay.y, r[DIM + 2 * p + 1]));
            }
        }
    }
}

// Only the diagonal of the reduced density matrix: rho_xx = sum |psi_x|^2.
template <int MASK>
__device__ __forceinline__ void rho_diag_partial(const double2 (&a)[16], double (&r)[1 << popc4(MASK)])
{
    constexpr int NB = popc4(MASK), DIM = 1 << NB, NG = 16 >> NB, REST = (~MASK) & 15;
#pragma unroll
    for (int i = 0; i < DIM; ++i) r[i] = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int x = 0; x < DIM; ++x) {
            const double2 ax = a[dep4(x, MASK) | dep4(g, REST)];
            r[x] = fma(ax.x, ax.x, fma(ax.y, ax.y, r[x]));
        }
}

// Index bits of register slot e on the register bits in MASK (the inverse of
// dep4): bit j of the result is the j-th set bit of MASK in e.
__host__ __device__ constexpr int ext4(int e, int mask)
{
    int out = 0, k = 0;
    for (int b = 0; b < 4; ++b)
        if (mask >> b & 1) {
            if (e >> b & 1) out |= 1 << k;
            ++k;
        }
    return out;
}

// A diagonal operator on the register bits in MASK (its diagonal read from
// the column-major matrix M): one factor per slot, real or complex.
template <int MASK>
__device__ __forceinline__ void apply_diag_op(const double2 (&a)[16], double2 (&y)[16], const double2 *__restrict__ M,
                                              bool real)
{
    constexpr int DIM = 1 << popc4(MASK);
    if (real) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const double f = M[ext4(e, MASK) * (DIM + 1)].x;
            y[e] = make_double2(f * a[e].x, f * a[e].y);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) y[e] = cmul(M[ext4(e, MASK) * (DIM + 1)], a[e]);
    }
}

// Tr(G rho) for Hermitian G (row-major) and rho packed as by rho_partial:
// sum_x G_xx rho_xx + 2 sum_{x<y} Re(G_xy conj(rho_xy)).
template <int DIM>
__device__ __forceinline__ double gram_weight(const double2 *__restrict__ G, const double (&r)[DIM * DIM])
{
    double w = 0.0;
#pragma unroll
    for (int x = 0; x < DIM; ++x) w = fma(G[x * DIM + x].x, r[x], w);
    int p = 0;
#pragma unroll
    for (int x = 0; x < DIM; ++x)
#pragma unroll
        for (int y = x + 1; y < DIM; ++y, ++p) {
            const double2 g = G[x * DIM + y];
            w = fma(2.0 * g.x, r[DIM + 2 * p], w);
            w = fma(2.0 * g.y, r[DIM + 2 * p + 1], w);
        }
    return w;
}

// A channel on the register bits in MASK.  The drawn operator is the
// smallest index i whose running sum of weights (taken in index order)
// exceeds u W, W the sum of all weights, or the last positive weight if
// rounding leaves none; a mixed-unitary channel's unitary is applied as
// stored, a general Kraus operator is divided by the square root of its
// weight.  A mixed-unitary channel stores the running sums themselves (the
// same sums, formed on the host), so its draw is a count of the sums not
// above u W; a general channel's weights Tr(K_i^dagger K_i rho_T) are formed
// twice (for W, then for the running sum) rather than kept in registers.
template <int MASK, bool WIDE>
__device__ __forceinline__ void traj_channel(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                             const double2 *__restrict__ M, double u, uint32_t log_tt,
                                             double *red, uint32_t wave, uint32_t wpt, uint32_t &flip)
{
    constexpr int DIM = 1 << popc4(MASK), D2 = DIM * DIM;
    const uint32_t nk = uni(op->nk);
    const bool mixed = uni(op->kind) == TOP_MIX;
    uint32_t j = 0;
    double wj = 1.0;
    const double2 *mats;
    if (mixed) {
        const double thr = u * M[nk - 1].x;
        for (uint32_t i = 0; i + 1 < nk; ++i) j += (M[i].x <= thr) ? 1u : 0u;
        mats = M + nk;
    } else {
        // weights Tr(G_i rho_T): from the diagonal of rho_T alone when every
        // Gram matrix is diagonal (amplitude damping), else from all of it
        double r[D2];
        if (uni(op->gdiag)) {
            double rd[DIM];
            rho_diag_partial<MASK>(x, rd);
            group_sum<DIM, WIDE>(rd, log_tt, red, wave, wpt, flip);
#pragma unroll
            for (int i = 0; i < D2; ++i) r[i] = (i < DIM) ? rd[i] : 0.0;
        } else {
            rho_partial<MASK>(x, r);
            group_sum<D2, WIDE>(r, log_tt, red, wave, wpt, flip);
        }
        double W = 0.0;
        for (uint32_t i = 0; i < nk; ++i) W += gram_weight<DIM>(M + i * D2, r);
        const double thr = u * W;
        double cum = 0.0, w_last = 0.0;
        bool found = false;
        uint32_t last = 0;
        for (uint32_t i = 0; i < nk; ++i) {
            const double wi = gram_weight<DIM>(M + i * D2, r);
            cum += wi;
            const bool take = !found && cum > thr;
            j = take ? i : j;
            wj = take ? wi : wj;
            found = found || take;
            last = (wi > 0.0) ? i : last;
            w_last = (wi > 0.0) ? wi : w_last;
        }
        if (!found) {
            j = last;
            wj = w_last;
        }
        mats = M + nk * D2;
    }
    // the drawn operator: per-slot factors when it is diagonal (the identity
    // of a mixed-unitary channel, the no-jump operator of damping), else the
    // dense product
    const uint32_t dmask = uni(op->dmask), rmask = uni(op->rmask);
    if (WIDE) {
        j = uni(j);              // one trajectory per wave: the operator's loads are scalar
        if ((dmask >> j) & 1u) apply_diag_op<MASK>(x, y, mats + j * D2, (rmask >> j) & 1u);
        else apply_mat<MASK, false>(x, y, mats + j * D2);
    } else {
        if (__all((dmask >> j) & 1u)) apply_diag_op<MASK>(x, y, mats + j * D2, __all((rmask >> j) & 1u));
        else apply_mat<MASK, false>(x, y, mats + j * D2);
    }
    if (!mixed) {
        const double s = 1.0 / sqrt(wj);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            y[e].x *= s;
            y[e].y *= s;
        }
    }
}

// A one-qubit channel whose draw needs only the coefficients inlined in its
// descriptor (TOp::inl), for trajectories of whole waves: the same draw and
// arithmetic as traj_channel, with the register bit a uniform runtime value,
// so one body serves every bit.  Returns false, having written nothing, when
// a general channel draws its non-diagonal operator (a jump, rare): the
// caller then runs traj_channel, which repeats the same draw.
template <bool WIDE>
__device__ __forceinline__ bool traj_channel_inline(const double2 (&x)[16], double2 (&y)[16], const TOp &op,
                                                    double u, uint32_t log_tt, double *red, uint32_t wave,
                                                    uint32_t wpt, uint32_t &flip)
{
    const uint32_t mask = uni(op.mask);
    const uint32_t bit = (mask & 1u) ? 0u : (mask & 2u) ? 1u : (mask & 4u) ? 2u : 3u;
    const bool mixed = uni(op.kind) == TOP_MIX;
    double f0, f1, s = 1.0;
    if (mixed) {
        const bool j = op.cf[0] <= u * op.cf[1];
        f0 = j ? op.cf[4] : op.cf[2];
        f1 = j ? op.cf[5] : op.cf[3];
    } else {
        double r[2];
        switch (mask) {
        case 1: rho_diag_partial<1>(x, r); break;
        case 2: rho_diag_partial<2>(x, r); break;
        case 4: rho_diag_partial<4>(x, r); break;
        default: rho_diag_partial<8>(x, r); break;
        }
        group_sum<2, WIDE>(r, log_tt, red, wave, wpt, flip);
        // gram_weight of a diagonal G: G_00 r_0, then + G_11 r_1 (its
        // off-diagonal terms add exact zeros)
        const double w0 = fma(op.cf[1], r[1], op.cf[0] * r[0]);
        const double w1 = fma(op.cf[3], r[1], op.cf[2] * r[0]);
        const double thr = u * (w0 + w1);
        // operator 0 unless the running sum passes u W only at operator 1
        // (or never, and the last positive weight is operator 1's)
        const bool jump = !(w0 > thr) && ((w0 + w1 > thr) || w1 > 0.0);
        if (jump) return false;
        f0 = op.cf[4];
        f1 = op.cf[5];
        s = 1.0 / sqrt(w0);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double f = ((uint32_t)e >> bit & 1u) ? f1 : f0;
        y[e] = make_double2(f * x[e].x, f * x[e].y);
    }
    if (!mixed) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            y[e].x *= s;
            y[e].y *= s;
        }
    }
    return true;
}

// Diagonal gates.  On register qubits only: one uniform factor per slot.
template <bool REAL>
__device__ __forceinline__ void traj_dreg(const double2 (&x)[16], double2 (&y)[16], const double2 *__restrict__ M)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double2 f = M[e];
        y[e] = REAL ? make_double2(f.x * x[e].x, f.x * x[e].y) : cmul(f, x[e]);
    }
}

// On thread qubits only: one factor per thread, from its thread bits.
__device__ __forceinline__ void traj_dthr(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                          const double2 *__restrict__ M, const TCtx &c)
{
    const uint32_t nd = uni(op->nd), q0 = uni(op->dq[0]) & 31u, q1 = uni(op->dq[1]) & 31u;
    const uint32_t tb = ((c.tl >> q0) & 1u) | ((nd > 1) ? (((c.tl >> q1) & 1u) << 1) : 0u);
    const double2 d0 = M[0], d1 = M[1];
    double2 d2 = d0, d3 = d1;
    if (nd > 1) {
        d2 = M[2];
        d3 = M[3];
    }
    const double2 f = (tb & 2u) ? ((tb & 1u) ? d3 : d2) : ((tb & 1u) ? d1 : d0);
#pragma unroll
    for (int e = 0; e < 16; ++e) y[e] = cmul(f, x[e]);
}

// One register qubit (bit MASK) and one thread qubit: two factors per thread,
// the slot's register bit picks one.
template <int MASK>
__device__ __forceinline__ void traj_dmix(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                          const double2 *__restrict__ M, const TCtx &c)
{
    const uint32_t tb = (c.tl >> (uni(op->dq[0]) & 31u)) & 1u;
    const double2 f0 = tb ? M[2] : M[0], f1 = tb ? M[3] : M[1];
#pragma unroll
    for (int e = 0; e < 16; ++e) y[e] = cmul((e & MASK) ? f1 : f0, x[e]);
}

// A register diagonal and a one-register, one-thread-qubit diagonal as one
// op: the 16 slot factors times the two factors the thread bit selects.
template <int MASK>
__device__ __forceinline__ void traj_drm(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                         const double2 *__restrict__ M, const TCtx &c)
{
    const uint32_t tb = (c.tl >> (uni(op->dq[0]) & 31u)) & 1u;
    const double2 f0 = tb ? M[18] : M[16], f1 = tb ? M[19] : M[17];
#pragma unroll
    for (int e = 0; e < 16; ++e) y[e] = cmul(cmul(M[e], (e & MASK) ? f1 : f0), x[e]);
}

// Two one-register, one-thread-qubit diagonals as one op: per slot, the
// factor the first's thread bit and register bit MASK select times the one
// the second's select (its register bit a uniform runtime value).
template <int MASK>
__device__ __forceinline__ void traj_dmix2(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                           const double2 *__restrict__ M, const TCtx &c)
{
    const uint32_t ta = (c.tl >> (uni(op->dq[0]) & 31u)) & 1u, tb = (c.tl >> (uni(op->dq[1]) & 31u)) & 1u;
    const uint32_t bit2 = uni(op->dmask);
    const double2 a0 = ta ? M[2] : M[0], a1 = ta ? M[3] : M[1];
    const double2 b0 = tb ? M[6] : M[4], b1 = tb ? M[7] : M[5];
#pragma unroll
    for (int e = 0; e < 16; ++e)
        y[e] = cmul(cmul((e & MASK) ? a1 : a0, ((uint32_t)e & bit2) ? b1 : b0), x[e]);
}

// A 2x2 complex matrix (column-major) on register bit MASK, in place.
template <int MASK>
__device__ __forceinline__ void mat1_inplace(double2 (&y)[16], const double2 *__restrict__ M)
{
    const double2 m00 = M[0], m10 = M[1], m01 = M[2], m11 = M[3];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (e & MASK) continue;
        const double2 a0 = y[e], a1 = y[e | MASK];
        double2 r0 = cmul(m00, a0), r1 = cmul(m10, a0);
        cmac<false>(r0, m01, a1);
        cmac<false>(r1, m11, a1);
        y[e] = r0;
        y[e | MASK] = r1;
    }
}

// nd one-qubit gates on register bits as one op (TOP_MATS).
__device__ __forceinline__ void traj_mats(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                          const double2 *__restrict__ M)
{
    const uint32_t nd = uni(op->nd), bits = uni(op->dmask);
    switch (bits & 3u) {
    case 0: apply_mat<1, false>(x, y, M); break;
    case 1: apply_mat<2, false>(x, y, M); break;
    case 2: apply_mat<4, false>(x, y, M); break;
    default: apply_mat<8, false>(x, y, M); break;
    }
    for (uint32_t j = 1; j < nd; ++j) {
        const double2 *Mj = M + 4 * j;
        switch ((bits >> (2 * j)) & 3u) {
        case 0: mat1_inplace<1>(y, Mj); break;
        case 1: mat1_inplace<2>(y, Mj); break;
        case 2: mat1_inplace<4>(y, Mj); break;
        default: mat1_inplace<8>(y, Mj); break;
        }
    }
}

template <bool WIDE>
__device__ __forceinline__ void traj_op(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                        const double2 *__restrict__ pool, const TCtx &c, double u, uint32_t log_tt,
                                        double *red, uint32_t wave, uint32_t wpt, uint32_t &flip)
{
    const uint32_t kind = uni(op->kind);
    const uint32_t mask = uni(op->mask);
    const double2 *M = pool + uni(op->mat);
    if (kind == TOP_MAT) {
        switch (mask | (uni(op->real) << 4)) {
#define VQD_TMAT(m)                                             \
    case m: apply_mat<m, false>(x, y, M); break;                \
    case 16 | m: apply_mat<m, true>(x, y, M); break;
        VQD_TMAT(1) VQD_TMAT(2) VQD_TMAT(3) VQD_TMAT(4) VQD_TMAT(5) VQD_TMAT(6) VQD_TMAT(7)
        VQD_TMAT(8) VQD_TMAT(9) VQD_TMAT(10) VQD_TMAT(11) VQD_TMAT(12) VQD_TMAT(13) VQD_TMAT(14)
        VQD_TMAT(15)
#undef VQD_TMAT
        default: break;
        }
    } else if (kind == TOP_DREG) {
        if (uni(op->real)) traj_dreg<true>(x, y, M);
        else traj_dreg<false>(x, y, M);
    } else if (kind == TOP_DTHR) {
        traj_dthr(x, y, op, M, c);
    } else if (kind == TOP_DMIX) {
        switch (mask) {
        case 1: traj_dmix<1>(x, y, op, M, c); break;
        case 2: traj_dmix<2>(x, y, op, M, c); break;
        case 4: traj_dmix<4>(x, y, op, M, c); break;
        default: traj_dmix<8>(x, y, op, M, c); break;
        }
    } else if (kind == TOP_MATS) {
        traj_mats(x, y, op, M);
    } else if (kind == TOP_DMIX2) {
        switch (mask) {
        case 1: traj_dmix2<1>(x, y, op, M, c); break;
        case 2: traj_dmix2<2>(x, y, op, M, c); break;
        case 4: traj_dmix2<4>(x, y, op, M, c); break;
        default: traj_dmix2<8>(x, y, op, M, c); break;
        }
    } else if (kind == TOP_DRM) {
        switch (mask) {
        case 1: traj_drm<1>(x, y, op, M, c); break;
        case 2: traj_drm<2>(x, y, op, M, c); break;
        case 4: traj_drm<4>(x, y, op, M, c); break;
        default: traj_drm<8>(x, y, op, M, c); break;
        }
    } else if (WIDE && uni(op->inl) == 2u && op->cf[0] > u * op->cf[1]) {
        // operator 0, the identity, is drawn (no running sum is <= u W);
        // the general path would multiply by factors of exactly 1
#pragma unroll
        for (int e = 0; e < 16; ++e) y[e] = x[e];
    } else if (WIDE && uni(op->inl) == 1u &&
               traj_channel_inline<WIDE>(x, y, *op, u, log_tt, red, wave, wpt, flip)) {
    } else {
        switch (mask) {
#define VQD_TCH(m) \
    case m: traj_channel<m, WIDE>(x, y, op, M, u, log_tt, red, wave, wpt, flip); break;
        VQD_TCH(1) VQD_TCH(2) VQD_TCH(4) VQD_TCH(8) VQD_TCH(3) VQD_TCH(5) VQD_TCH(6) VQD_TCH(9)
        VQD_TCH(10) VQD_TCH(12)
#undef VQD_TCH
        default: break;
        }
    }
}

// The uniforms of one trajectory, fetched in blocks: the LG = min(2^log_tt,
// 64) lanes of a trajectory inside a wave hold one block of LG consecutive
// channels (lane j channel base + j) and the next block is loaded one block
// ahead.  Channels are met in increasing order (the same order in every
// trajectory of the workgroup), so a channel's uniform is a lane shuffle.
struct UBlock {
    const double *row;   // this trajectory's uniforms
    uint32_t n_ch, lg, gl0, LG;
    uint32_t base;       // first channel of the current block
    double cur, nxt;

    __device__ __forceinline__ void start(const double *r, uint32_t nch, uint32_t log_tt)
    {
        row = r;
        n_ch = nch;
        LG = 1u << (log_tt < 6 ? log_tt : 6);
        const uint32_t lane = threadIdx.x & 63u;
        lg = lane & (LG - 1u);
        gl0 = lane & ~(LG - 1u);
        base = 0;
        cur = (lg < n_ch) ? row[lg] : 0.0;
        nxt = (LG + lg < n_ch) ? row[LG + lg] : 0.0;
    }

    template <bool WIDE>
    __device__ __forceinline__ double take(uint32_t ch)
    {
        if (ch >= base + LG) {           // workgroup-uniform
            cur = nxt;
            base += LG;
            const uint32_t k = base + LG + lg;
            nxt = (k < n_ch) ? row[k] : 0.0;
        }
        if (WIDE) {                      // one trajectory per wave: the lane is uniform
            const int src = (int)(ch - base);
            const uint64_t bits = __double_as_longlong(cur);
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)bits, src);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(bits >> 32), src);
            return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
        }
        return __shfl(cur, (int)(gl0 + (ch - base)));
    }
};

// A run of one-qubit channels with inline coefficients (TOp::grp), drawn
// with one reduction for trajectories of whole waves.  Damping members are
// diagonal when no jump is drawn and the mixed-unitary members leave the
// populations alone, so every damping draw's weights follow from the run's
// input populations p_e: with q_e^(k) = p_e times the no-jump Gram factors
// G0 of the damping members before member k, and C_k = sum_e q_e^(k), the
// state before member k is the input scaled by its no-jump factors over
// sqrt(C_k / C_0), so that member's weights are proportional to C_(k+1) for
// the no-jump operator and to D_k = sum_e q_e^(k) G1(e) for the jump.  The
// members are trace preserving (G0 + G1 = I, checked by the planner), so
// C_(k+1) + D_k = C_k: the reduction carries C_0 .. C_K only, and the draws
// compare C_(k+1) and C_k with u C_k.  The result is the input times every
// member's diagonal factors over sqrt(C_K): the member-by-member draws
// normalise by the weights as they form them, whose product is C_K.  When a
// damping member draws its jump, only the members before it are applied
// (over sqrt of the running sum before it) and their count is returned:
// the caller takes the rest one by one, from the member that jumped, which
// repeats its draw.  Returns the number of members applied (0: nothing
// written).
__device__ __forceinline__ uint32_t member_bit(uint32_t mask)
{
    return (mask & 1u) ? 0u : (mask & 2u) ? 1u : (mask & 4u) ? 2u : 3u;
}

// One damping member of a run, register bit MASK: this thread's part of
// C_(k+1) = sum_e q_e G0(e), from the populations with the bit clear (s0)
// and set (s1), each summed as a tree; then q_e *= G0(e).
template <int MASK>
__device__ __forceinline__ void damp_member(double (&q)[16], double g00, double g01, double &cs)
{
    double h[2][8];
    int n0 = 0, n1 = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (e & MASK) h[1][n1++] = q[e];
        else h[0][n0++] = q[e];
    }
    double s[2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
        s[b] = ((h[b][0] + h[b][1]) + (h[b][2] + h[b][3])) + ((h[b][4] + h[b][5]) + (h[b][6] + h[b][7]));
    cs = fma(g01, s[1], g00 * s[0]);
#pragma unroll
    for (int e = 0; e < 16; ++e) q[e] *= (e & MASK) ? g01 : g00;
}

template <bool WIDE>
__device__ __forceinline__ uint32_t traj_group(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ op,
                                           uint32_t k, UBlock &ub, uint32_t &next_ch, uint32_t log_tt,
                                           double *red, uint32_t wave, uint32_t wpt, uint32_t &flip)
{
    constexpr int NK = (int)kTrajGroupKraus;
    double u[kTrajGroupMax];
#pragma unroll
    for (uint32_t i = 0; i < kTrajGroupMax; ++i) {
        u[i] = 0.0;
        if (i < k) u[i] = ub.take<WIDE>(next_ch++);
    }
    double q[16], r[NK + 1];
#pragma unroll
    for (int e = 0; e < 16; ++e) q[e] = fma(x[e].x, x[e].x, x[e].y * x[e].y);
    r[0] = (((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]))) +
           (((q[8] + q[9]) + (q[10] + q[11])) + ((q[12] + q[13]) + (q[14] + q[15])));
#pragma unroll
    for (int j = 1; j <= NK; ++j) r[j] = 0.0;
    uint32_t kk = 0;
#pragma unroll
    for (uint32_t i = 0; i < kTrajGroupMax; ++i) {
        if (i < k && uni(op[i].kind) == TOP_KRAUS) {
            const double g00 = op[i].cf[0], g01 = op[i].cf[1];
            double cs;
            switch (uni(op[i].mask)) {
            case 1: damp_member<1>(q, g00, g01, cs); break;
            case 2: damp_member<2>(q, g00, g01, cs); break;
            case 4: damp_member<4>(q, g00, g01, cs); break;
            default: damp_member<8>(q, g00, g01, cs); break;
            }
#pragma unroll
            for (int j = 0; j < NK; ++j) r[j + 1] += (kk == (uint32_t)j) ? cs : 0.0;
            ++kk;
        }
    }
    group_sum<NK + 1, WIDE>(r, log_tt, red, wave, wpt, flip);
    // members before the first drawn jump (all of them when none is) are
    // applied: their factors, and the normalisation 1 / sqrt(C_kk) of the kk
    // damping members among them (none: 1)
    bool jump = false;
    uint32_t used = k;
    double last = 1.0, f0b[4] = {1.0, 1.0, 1.0, 1.0}, f1b[4] = {1.0, 1.0, 1.0, 1.0};
    kk = 0;
#pragma unroll
    for (uint32_t i = 0; i < kTrajGroupMax; ++i) {
        if (i < k && !jump) {
            const TOp &m = op[i];
            const uint32_t bit = member_bit(uni(m.mask));
            double f0, f1;
            if (uni(m.kind) == TOP_MIX) {
                const bool j = m.cf[0] <= u[i] * m.cf[1];
                f0 = j ? m.cf[4] : m.cf[2];
                f1 = j ? m.cf[5] : m.cf[3];
            } else {
                double tot = r[0], cw = r[1];
#pragma unroll
                for (int j = 1; j < NK; ++j) {
                    tot = (kk == (uint32_t)j) ? r[j] : tot;
                    cw = (kk == (uint32_t)j) ? r[j + 1] : cw;
                }
                const double dw = tot - cw, thr = u[i] * tot;
                jump = !(cw > thr) && (tot > thr || dw > 0.0);
                f0 = jump ? 1.0 : m.cf[4];
                f1 = jump ? 1.0 : m.cf[5];
                used = jump ? i : used;
                last = jump ? last : cw;
                kk += jump ? 0u : 1u;
            }
#pragma unroll
            for (uint32_t b = 0; b < 4; ++b) {
                f0b[b] *= (bit == b) ? f0 : 1.0;
                f1b[b] *= (bit == b) ? f1 : 1.0;
            }
        }
    }
    if (used == 0) return 0;
    const double s = (kk == 0) ? 1.0 : 1.0 / sqrt(last);
    double lo[4], hi[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        lo[v] = ((v & 1) ? f1b[0] : f0b[0]) * ((v & 2) ? f1b[1] : f0b[1]) * s;
        hi[v] = ((v & 1) ? f1b[2] : f0b[2]) * ((v & 2) ? f1b[3] : f0b[3]);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double f = lo[e & 3] * hi[e >> 2];
        y[e] = make_double2(f * x[e].x, f * x[e].y);
    }
    return used;
}

// One step of a phase's op list, x -> y: a marked run as one draw when the
// trajectory is whole waves and no member jumps, else the op at oi alone.
// Returns the index of the next op.
template <bool WIDE>
__device__ __forceinline__ uint32_t traj_step(const double2 (&x)[16], double2 (&y)[16], const TOp *__restrict__ ops,
                                              uint32_t oi, uint32_t oe, const double2 *__restrict__ pool,
                                              const TCtx &c, UBlock &ub, uint32_t &next_ch, uint32_t log_tt,
                                              double *red, uint32_t wave, uint32_t wpt, uint32_t &flip)
{
    const TOp *op = ops + oi;
    if (WIDE && uni(op->inl) == 2u && oi + 1 < oe && uni(op[1].inl) == 2u) {
        // two identity-first channels in a row: when both draw operator 0
        // (the common case) the state is copied once
        const uint32_t base = ub.base, ch = next_ch;
        const double cur = ub.cur, nxt = ub.nxt;
        const double u0 = ub.take<WIDE>(next_ch++), u1 = ub.take<WIDE>(next_ch++);
        if (op->cf[0] > u0 * op->cf[1] && op[1].cf[0] > u1 * op[1].cf[1]) {
#pragma unroll
            for (int e = 0; e < 16; ++e) y[e] = x[e];
            return oi + 2;
        }
        ub.base = base;
        ub.cur = cur;
        ub.nxt = nxt;
        next_ch = ch;
    }
    if (WIDE) {
        const uint32_t k = uni(op->grp);
        if (k > 1u) {
            const uint32_t base = ub.base, ch = next_ch;
            const double cur = ub.cur, nxt = ub.nxt;
            const uint32_t used = traj_group<WIDE>(x, y, op, k, ub, next_ch, log_tt, red, wave, wpt, flip);
            if (used == k) return oi + k;
            // the rest of the run one by one, from the same uniforms: the
            // member that drew its jump comes next (at oi itself when it is
            // the first, and nothing has been written)
            ub.base = base;
            ub.cur = cur;
            ub.nxt = nxt;
            next_ch = ch + used;
            if (used) return oi + used;
        }
    }
    double u = 0.0;
    if (is_channel(uni(op->kind))) u = ub.take<WIDE>(next_ch++);
    traj_op<WIDE>(x, y, op, pool, c, u, log_tt, red, wave, wpt, flip);
    return oi + 1;
}

// Orders one wave's LDS accesses for the compiler; the hardware executes a
// wave's LDS instructions in issue order.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One batch of trajectories.  Workgroup g of the persistent loop holds
// blockDim / 2^log_tt trajectories; group grp's threads are tid >> log_tt.
template <bool WIDE>
__global__ void __launch_bounds__(512)
k_traj(const TPhase *__restrict__ phases, uint32_t n_phases, const TOp *__restrict__ ops,
       const double2 *__restrict__ pool, uint32_t n, uint32_t log_tt, uint32_t n_ch,
       const double *__restrict__ U, uint64_t T, double *__restrict__ z_out, double *__restrict__ norm_out,
       double *__restrict__ state_out)
{
    extern __shared__ double2 lds[];
    const uint32_t tid = threadIdx.x;
    const uint32_t TT = 1u << log_tt;
    const uint32_t tpw = blockDim.x >> log_tt;
    const uint32_t grp = tid >> log_tt, tt = tid & (TT - 1u);
    const uint32_t wave = uni(tid >> 6), wpt = WIDE ? (TT >> 6) : 1u;
    double *red = reinterpret_cast<double *>(lds + (size_t)blockDim.x * 16);
    double2 *xl = lds + (size_t)grp * TT * 16;
    // LDS index of amplitude t | s (thread part t, slot part s) is
    // swz(t) ^ swz(s) ^ gx: the swizzle is xor-linear, so the slot part is
    // workgroup-uniform.  gx permutes the low index bits by trajectory so
    // that lanes of different trajectories in one wave spread over the banks.
    const uint32_t gx = (grp << log_tt) & 7u;
    const uint64_t n_groups = (T + tpw - 1) / tpw;
    const uint32_t dim = 1u << n;
    uint32_t flip = 0;
    // A trajectory inside one wave owns its LDS region alone: its exchanges
    // need no workgroup barrier, only the wave's own (in-order) LDS accesses.
    const bool shared_tile = WIDE && wpt > 1;

    for (uint64_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const uint64_t traj = g * tpw + grp;
        const bool active = traj < T;
        UBlock ub;
        ub.start(U + (active ? traj : T - 1) * (uint64_t)n_ch, n_ch, log_tt);
        uint32_t next_ch = 0;
        double2 a[16], b[16];
        TCtx c;
        for (uint32_t ph = 0; ph < n_phases; ++ph) {
            const TPhase *H = phases + ph;
#pragma unroll
            for (int r = 0; r < 4; ++r) c.rl[r] = 1u << (uni(H->reg_q[r]) & 31u);
            c.tl = traj_thread_bits(H, tt);
            if (ph == 0) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    a[e] = make_double2(((c.tl | slot_l(c.rl, e)) == 0u) ? 1.0 : 0.0, 0.0);
            } else {
                const uint32_t lt = swz(c.tl) ^ gx;
#pragma unroll
                for (int e = 0; e < 16; ++e) a[e] = xl[lt ^ uni(H->lds_slot[e])];
                // the barrier that lets the next exchange overwrite this one:
                // a general channel's reduction in the phase is one already
                if (!shared_tile) wave_lds_sync();
                else if (!(uni(H->flags) & kTPhaseReduces)) __syncthreads();
            }
            const uint32_t oe = uni(H->op_end);
            uint32_t oi = uni(H->op_begin);
            while (oi < oe) {
                oi = traj_step<WIDE>(a, b, ops, oi, oe, pool, c, ub, next_ch, log_tt, red, wave, wpt, flip);
                if (oi < oe) {
                    oi = traj_step<WIDE>(b, a, ops, oi, oe, pool, c, ub, next_ch, log_tt, red, wave, wpt, flip);
                } else {
#pragma unroll
                    for (int e = 0; e < 16; ++e) a[e] = b[e];
                }
            }
            if (ph + 1 < n_phases) {
                const uint32_t lt = swz(traj_thread_bits(H, tt)) ^ gx;
#pragma unroll
                for (int e = 0; e < 16; ++e) xl[lt ^ uni(H->lds_slot[e])] = a[e];
                if (shared_tile) __syncthreads();
                else wave_lds_sync();
            }
        }

        // read-out: <Z_q> for q < n in r[q], the squared norm in r[15]
        double r[kTrajRed];
#pragma unroll
        for (int i = 0; i < kTrajRed; ++i) r[i] = 0.0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t xi = c.tl | slot_l(c.rl, e);
            const double p = fma(a[e].x, a[e].x, a[e].y * a[e].y);
            r[15] += p;
#pragma unroll
            for (int q = 0; q < kTrajMaxQubits; ++q) r[q] += ((xi >> q) & 1u) ? -p : p;
        }
        group_sum<kTrajRed, WIDE>(r, log_tt, red, wave, wpt, flip);
        if (active) {
            if (tt == 0) {
                for (uint32_t q = 0; q < n; ++q) z_out[traj * n + q] = r[q];
                if (norm_out) norm_out[traj] = r[15];
            }
            if (state_out) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const uint32_t xi = c.tl | slot_l(c.rl, e);
                    if (xi < dim) {
                        state_out[2 * (traj * dim + xi)] = a[e].x;
                        state_out[2 * (traj * dim + xi) + 1] = a[e].y;
                    }
                }
            }
        }
    }
}

// Column j of the T x m row-major samples: mean, then the sum of squared
// deviations from it, each summed per thread in row order and then over the
// threads in a fixed tree.
constexpr int kStatThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kStatThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

__global__ void __launch_bounds__(kStatThreads)
k_traj_stats(const double *__restrict__ x, uint64_t T, uint32_t m, double *__restrict__ mean,
             double *__restrict__ sem)
{
    __shared__ double sh[kStatThreads];
    const uint32_t j = blockIdx.x;
    double s = 0.0;
    for (uint64_t t = threadIdx.x; t < T; t += kStatThreads) s += x[t * m + j];
    const double mu = block_sum(s, sh) / (double)T;
    double q = 0.0;
    for (uint64_t t = threadIdx.x; t < T; t += kStatThreads) {
        const double d = x[t * m + j] - mu;
        q = fma(d, d, q);
    }
    const double Q = block_sum(q, sh);
    if (threadIdx.x == 0) {
        mean[j] = mu;
        sem[j] = (T > 1) ? sqrt(Q / (double)(T - 1)) / sqrt((double)T) : INFINITY;
    }
}

}  // namespace

int launch_traj(const TPhase *phases, uint32_t n_phases, const TOp *ops, const double2 *pool, int n,
                int n_eff, uint32_t n_ch, const double *U, uint64_t T, double *z_out, double *norm_out,
                double *state_out, hipStream_t stream)
{
    if (T == 0) return VQD_OK;
    const uint32_t log_tt = (uint32_t)(n_eff - 4);
    const uint32_t threads = (log_tt == 9) ? 512u : 256u;
    const size_t lds = size_t(threads) * 16 * sizeof(double2) + size_t(2 * kTrajMaxWaves) * kTrajRed * sizeof(double);
    const bool wide = log_tt >= 6;
    const void *kfn = wide ? (const void *)k_traj<true> : (const void *)k_traj<false>;
    static bool attr_set = false;
    static int n_cu = 0;
    if (!attr_set) {
        VQD_HIP(hipFuncSetAttribute((const void *)k_traj<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024));
        VQD_HIP(hipFuncSetAttribute((const void *)k_traj<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024));
        int dev_id = 0;
        VQD_HIP(hipGetDevice(&dev_id));
        VQD_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id));
        attr_set = true;
    }
    int per_cu = 0;
    VQD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, (int)threads, lds));
    if (per_cu < 1) per_cu = 1;
    const uint32_t tpw = threads >> log_tt;
    const uint64_t n_groups = (T + tpw - 1) / tpw;
    uint64_t grid = (uint64_t)per_cu * (uint64_t)n_cu;
    if (grid > n_groups) grid = n_groups;
    if (wide)
        hipLaunchKernelGGL(k_traj<true>, dim3((uint32_t)grid), dim3(threads), lds, stream, phases, n_phases, ops,
                           pool, (uint32_t)n, log_tt, n_ch, U, T, z_out, norm_out, state_out);
    else
        hipLaunchKernelGGL(k_traj<false>, dim3((uint32_t)grid), dim3(threads), lds, stream, phases, n_phases, ops,
                           pool, (uint32_t)n, log_tt, n_ch, U, T, z_out, norm_out, state_out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int launch_traj_stats(const double *x, uint64_t T, int m, double *mean, double *sem, hipStream_t stream)
{
    if (m <= 0) return VQD_OK;
    hipLaunchKernelGGL(k_traj_stats, dim3((uint32_t)m), dim3(kStatThreads), 0, stream, x, T, (uint32_t)m, mean,
                       sem);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

}  // namespace vqd
