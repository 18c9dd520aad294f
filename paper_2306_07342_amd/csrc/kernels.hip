// gfx950 kernels of the vqd library.
//
// * k_pass     -- one HBM pass over the vectorised density matrix applying a
//                 planned sequence of register phases (see vqd_internal.h).
// * k_init     -- |b><b| and the product-diagonal (thermal) initial states.
// * k_purity / k_diag / k_zz / k_pauli -- read-out reductions (wave shuffles,
//                 then one partial per workgroup, then a fixed-order second
//                 stage, so results are deterministic).
#include <hip/hip_runtime.h>

#include <mutex>

#include "vqd_internal.h"
#include "dev_common.h"

namespace vqd {

namespace {

constexpr int kThreads = 256;

// Flip-pattern matrix: y[i] = sum_x W[x][i] a[i ^ flip(x)], flip(x) flipping
// the row and the column bit of the same qubit(s).  Pauli channels, amplitude
// damping and their products with diagonal ops have this form.
template <int MASK>
__host__ __device__ constexpr int slot_flip(int x)
{
    return MASK == 5 ? (x ? 5 : 0) : MASK == 10 ? (x ? 10 : 0) : ((x & 1) ? 5 : 0) | ((x & 2) ? 10 : 0);
}

template <int MASK, bool REAL>
__device__ __forceinline__ void apply_xor(const double2 (&a)[16], double2 (&y)[16], const double2 *__restrict__ M)
{
    constexpr int NB = popc4(MASK), DIM = 1 << NB, NG = 16 >> NB, REST = (~MASK) & 15;
    constexpr int NX = (MASK == 15) ? 4 : 2;
#pragma unroll
    for (int x = 0; x < NX; ++x) {
        double2 w[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) w[i] = coef<REAL>(M, x * DIM + i);
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int so = dep4(i, MASK) | dep4(g, REST), si = so ^ slot_flip<MASK>(x);
                if (x == 0) {
                    y[so].x = w[i].x * a[si].x;
                    y[so].y = w[i].x * a[si].y;
                    if (!REAL) {
                        y[so].x = fma(-w[i].y, a[si].y, y[so].x);
                        y[so].y = fma(w[i].y, a[si].x, y[so].y);
                    }
                } else {
                    cmac<REAL>(y[so], w[i], a[si]);
                }
            }
    }
}

template <bool REAL>
__device__ __forceinline__ double2 fmul(const double2 m, const double2 x)
{
    return REAL ? make_double2(m.x * x.x, m.x * x.y) : cmul(m, x);
}

// Element-wise factors indexed by the register slot.
template <bool REAL>
__device__ __forceinline__ void apply_diag(const double2 (&a)[16], double2 (&y)[16], const double2 *__restrict__ M)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) y[e] = fmul<REAL>(coef<REAL>(M, e), a[e]);
}

// Per-phase, per-thread context of the op loop.
struct Ctx {
    uint32_t gb;        // global index bits of the tile (workgroup-uniform)
    uint32_t tl;        // local index bits from the thread id
    uint32_t rl[4];     // local bit of register bit b
};

// Table index of a runtime diagonal: gathered bit j comes from the tile's
// group bits (uniform) or from local index bits of `loc`.
// Branch-free over the four entries, so that the descriptor fields arrive in
// one batch of scalar loads rather than one load-and-wait per bit.
__device__ __forceinline__ uint32_t rt_index(const KOp *__restrict__ op, uint32_t nb, uint32_t gb,
                                             uint32_t loc)
{
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t lp = uni(op->lpos[j]), gp = uni(op->gpos[j]);
        const uint32_t b = (lp == kNotLocal) ? ((gb >> (gp & 31u)) & 1u) : ((loc >> (lp & 31u)) & 1u);
        r |= (((uint32_t)j < nb) ? b : 0u) << j;
    }
    return r;
}

// Element-wise factors from an LDS table indexed by global bits (see RtMode).
template <uint32_t MODE, bool REAL>
__device__ __forceinline__ void apply_diag_rt(const double2 (&a)[16], double2 (&y)[16], const KOp *__restrict__ op,
                                              const double2 *T, const Ctx &c)
{
    const uint32_t nb = uni(op->nbits);
    if (MODE == RT_NONE) {
        const double2 f = T[rt_index(op, nb, c.gb, c.tl)];
#pragma unroll
        for (int e = 0; e < 16; ++e) y[e] = fmul<REAL>(f, a[e]);
    } else if (MODE == RT_PAIR_A || MODE == RT_PAIR_B) {
        constexpr int R = (MODE == RT_PAIR_A) ? 0 : 1;
        const uint32_t base = 4 * rt_index(op, nb, c.gb, c.tl);
        double2 f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = T[base + k];
#pragma unroll
        for (int e = 0; e < 16; ++e) y[e] = fmul<REAL>(f[((e >> R) & 1) | (((e >> (R + 2)) & 1) << 1)], a[e]);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            y[e] = fmul<REAL>(T[rt_index(op, nb, c.gb, c.tl | slot_l(c.rl, e))], a[e]);
    }
}

// Global bits of tile t (workgroup-uniform).  Amplitude indices fit in 32
// bits (2n <= 32); 32-bit index arithmetic keeps the per-slot offsets that
// stay live across the tile loop in half as many scalar registers.
__device__ __forceinline__ uint32_t group_base(const KPass *__restrict__ P, uint32_t t, uint32_t ngb,
                                               bool xcd)
{
    if (xcd) {
        // workgroup b runs on XCD b % 8: the tiles that differ in the lowest
        // group bits (and share cache lines) are given to one XCD
        const uint32_t x = t & 7u, s = t >> 3;
        t = (s & 7u) | (x << 3) | ((s >> 3) << 6);
    }
    uint32_t g = 0;
    for (uint32_t i = 0; i < ngb; ++i) g |= ((t >> i) & 1u) << uni(P->group_gpos[i]);
    return g;
}

// Hermitian mode: launched tile t is the group pair (i, j), i <= j < N = 2^m.
// The c lowest group bits split 128-byte lines between tiles, so the pairs
// are launched in blocks: i = I 2^c + a, j = J 2^c + b (a, b < 2^c), the
// blocks I <= J < 2^(m-c) enumerated by folding row I with row NB-1-I of
// the upper triangle (NB + 1 blocks per fold), a block's 4^c members s =
// min(8, blocks) launch indices apart (one XCD, one round of the persistent
// grid; no padding when a pass has fewer than 8 blocks).  The
// tile's base holds i in the m row group bits and j in the m column group
// bits, its mirror's base the other way round.  Padding blocks and members
// with a > b of a block with I = J are not stored.
struct HermTile {
    uint32_t gb, gbm;    // load base and its mirror (the layout the pass loads)
    uint32_t gbs, gbms;  // store base and its mirror (the layout the pass stores)
    bool mirror;         // i < j: the tile's conjugate transpose is stored too
    bool valid;          // a tile of the upper triangle (stored)
};

__device__ __forceinline__ HermTile herm_tile(const KPass *__restrict__ P, uint32_t t, uint32_t ngb,
                                              uint32_t herm)
{
    const uint32_t m = ngb >> 1, c = (herm >> kHermLineShift) & 3u, st = (herm >> kHermStrideShift) & 15u;
    const uint32_t NB = 1u << (m - c), NBB = NB * (NB + 1) / 2;
    const uint32_t q0 = (st == 8u) ? t >> 3 : t / st, lo = t - q0 * st;
    const uint32_t k = q0 & ((1u << (2 * c)) - 1u), hi = q0 >> (2 * c);
    const uint32_t beta = hi * st + lo;
    uint32_t I = 0, J = 0;
    if (NB > 1) {
        const uint32_t a = beta / (NB + 1), b = beta - a * (NB + 1);
        if (b < NB - a) {
            I = a;
            J = a + b;
        } else {
            I = NB - 1 - a;
            J = I + (b - (NB - a));
        }
    }
    const uint32_t ma = k & ((1u << c) - 1u), mb = k >> c;
    const uint32_t i = (I << c) | ma, j = (J << c) | mb;
    HermTile h{0u, 0u, 0u, 0u, i != j, beta < NBB && (I < J || ma <= mb)};
    for (uint32_t q = 0; q < m; ++q) {
        const uint32_t gr = uni(P->group_gpos[q]), gc = uni(P->group_gpos[m + q]);
        const uint32_t sr = uni(P->out_gpos[q]), sc = uni(P->out_gpos[m + q]);
        const uint32_t bi = (i >> q) & 1u, bj = (j >> q) & 1u;
        h.gb |= (bi << gr) | (bj << gc);
        h.gbm |= (bj << gr) | (bi << gc);
        h.gbs |= (bi << sr) | (bj << sc);
        h.gbms |= (bj << sr) | (bi << sc);
    }
    return h;
}


// Local and global index bits contributed by the thread id in phase H.
// Thread-id bits at or above nthr are zero (tid < 2^nthr) and the unused
// descriptor entries are zero-filled, so the loops run over the fixed
// maximum without branches.
__device__ __forceinline__ void thread_bits(const KPhase *__restrict__ H, uint32_t tid, uint32_t nthr,
                                            uint32_t &tl, uint32_t &tg)
{
    (void)nthr;
    tl = 0;
    tg = 0;
#pragma unroll
    for (uint32_t i = 0; i < (uint32_t)kMaxThreadBits; ++i) {
        const uint32_t b = (tid >> i) & 1u;
        tl |= b << (uni(H->thr_local[i]) & 31u);
        tg |= b << (uni(H->thr_gpos[i]) & 31u);
    }
}

// Fully unrolled over the fixed maximum so that the descriptor reads are
// scalar loads: a vector load here would make the compiler wait for the
// outstanding prefetch of the next tile.
__device__ __forceinline__ uint32_t thread_local_bits(const KPhase *__restrict__ H, uint32_t tid,
                                                      uint32_t nthr)
{
    (void)nthr;
    uint32_t tl = 0;
#pragma unroll
    for (uint32_t i = 0; i < (uint32_t)kMaxThreadBits; ++i) tl |= ((tid >> i) & 1u) << (uni(H->thr_local[i]) & 31u);
    return tl;
}

// Global index part of register slot e (precomputed by the planner).
__device__ __forceinline__ uint32_t slot_g(const KPhase *__restrict__ H, int e) { return uni(H->g_slot[e]); }

// Hermitian mode: the conjugate of the tile's amplitude in slot e goes to
// the transposed index (row and column bits exchanged): the mirrored group
// base, the transposed slot bits and the thread's transposed bits (in
// `lane`).  The mirror tile is never computed itself.
__device__ __forceinline__ void store_mirror(double2 *lane, uint32_t gbm, const KPhase *__restrict__ H,
                                             const double2 (&a)[16])
{
#pragma unroll
    for (int e = 0; e < 16; ++e) lane[gbm | uni(H->gm_slot[e])] = make_double2(a[e].x, -a[e].y);
}

// The previous pass's group pair of an amplitude: i collects its bits at
// that pass's row group positions, j at the column positions (in the layout
// that pass stored, which is the one this pass loads).  Index bits
// come from the thread (fixed per pass), the register slot and the tile's
// group base, which occupy disjoint positions, so i and j are ORs of parts.
struct HalfIn {
    uint32_t it, jt;           // thread parts
    uint32_t m;                // group pairs of the previous pass
    const KPass *Pp;           // the previous pass
};

__device__ __forceinline__ void pair_of(const KPass *__restrict__ Pp, uint32_t m, uint32_t x, uint32_t &i,
                                        uint32_t &j)
{
    i = 0;
    j = 0;
    for (uint32_t k = 0; k < m; ++k) {
        i |= ((x >> (uni(Pp->out_gpos[k]) & 31u)) & 1u) << k;
        j |= ((x >> (uni(Pp->out_gpos[m + k]) & 31u)) & 1u) << k;
    }
}

__device__ __forceinline__ HalfIn half_in(const KPass *__restrict__ P, uint32_t tg0)
{
    HalfIn h;
    h.Pp = P - 1;
    h.m = uni(h.Pp->n_group_bits) >> 1;
    pair_of(h.Pp, h.m, tg0, h.it, h.jt);
    return h;
}

// Hermitian-mode loads of one tile: slot e from its own index, or, where the
// previous pass did not store it (its group pair there had i > j), the
// conjugate of the amplitude at the transposed index.  The choice depends on
// bits of qubits outside every Hermitian tile's forced low qubits, so the
// lanes of one coalesced segment make the same choice.
__device__ __forceinline__ void load_herm(double2 (&v)[16], const double2 *__restrict__ lane,
                                          const double2 *__restrict__ lane_m, const HermTile &ht,
                                          const KPass *__restrict__ P, const KPhase *__restrict__ H0,
                                          uint32_t herm, const HalfIn &hin)
{
    if (!(herm & kHermHalfIn)) {
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = lane[ht.gb | uni(H0->g_slot[e])];
        return;
    }
    uint32_t ig, jg;
    pair_of(hin.Pp, hin.m, ht.gb, ig, jg);
    const uint32_t i0 = ig | hin.it, j0 = jg | hin.jt;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const uint32_t u = ht.gb | uni(H0->g_slot[e]), um = ht.gbm | uni(H0->gm_slot[e]);
        const uint32_t i = i0 | uni(P->hi_slot[e]), j = j0 | uni(P->hj_slot[e]);
        const bool tr = i > j;
        // one load from the selected address (not two loads and a select)
        const double2 w = *(tr ? lane_m + um : lane + u);
        v[e] = make_double2(w.x, tr ? -w.y : w.y);
    }
}

// One op: y = op(x).
__device__ __forceinline__ void apply_op(const double2 (&x)[16], double2 (&y)[16], const KOp *__restrict__ op,
                                         const double2 *__restrict__ mats, const double2 *lds_rt, const Ctx &c)
{
    const uint32_t kind = uni(op->kind);
    const uint32_t sel = uni(op->opmask) | (uni(op->real) << 4);
    const double2 *M = mats + uni(op->mat);
    if (kind == KOP_MAT) {
        switch (sel) {
        case 5: apply_mat<5, false>(x, y, M); break;
        case 10: apply_mat<10, false>(x, y, M); break;
        case 15: apply_mat<15, false>(x, y, M); break;
        case 7: apply_mat<7, false>(x, y, M); break;
        case 16 | 5: apply_mat<5, true>(x, y, M); break;
        case 16 | 10: apply_mat<10, true>(x, y, M); break;
        case 16 | 15: apply_mat<15, true>(x, y, M); break;
        default: apply_mat<7, true>(x, y, M); break;
        }
    } else if (kind == KOP_XOR) {
        switch (sel) {
        case 5: apply_xor<5, false>(x, y, M); break;
        case 10: apply_xor<10, false>(x, y, M); break;
        case 15: apply_xor<15, false>(x, y, M); break;
        case 16 | 5: apply_xor<5, true>(x, y, M); break;
        case 16 | 10: apply_xor<10, true>(x, y, M); break;
        default: apply_xor<15, true>(x, y, M); break;
        }
    } else if (kind == KOP_DIAG) {
        if (sel & 16) apply_diag<true>(x, y, M);
        else apply_diag<false>(x, y, M);
    } else if (kind == KOP_PTM) {
        if (uni(op->opmask) == 5) apply_ptm<5>(x, y, M);
        else apply_ptm<10>(x, y, M);
    } else {
        const double2 *T = lds_rt + uni(op->mat);
        switch (uni(op->mode) | (sel & 16)) {
        case RT_NONE: apply_diag_rt<RT_NONE, false>(x, y, op, T, c); break;
        case RT_PAIR_A: apply_diag_rt<RT_PAIR_A, false>(x, y, op, T, c); break;
        case RT_PAIR_B: apply_diag_rt<RT_PAIR_B, false>(x, y, op, T, c); break;
        case RT_GENERIC: apply_diag_rt<RT_GENERIC, false>(x, y, op, T, c); break;
        case 16 | RT_NONE: apply_diag_rt<RT_NONE, true>(x, y, op, T, c); break;
        case 16 | RT_PAIR_A: apply_diag_rt<RT_PAIR_A, true>(x, y, op, T, c); break;
        case 16 | RT_PAIR_B: apply_diag_rt<RT_PAIR_B, true>(x, y, op, T, c); break;
        default: apply_diag_rt<RT_GENERIC, true>(x, y, op, T, c); break;
        }
    }
}

// The phase's ops, two at a time between a and b so that no op copies its
// results back into its input registers; an odd count ends with one copy.
__device__ __forceinline__ void apply_ops(double2 (&a)[16], const KPhase *__restrict__ H,
                                          const KOp *__restrict__ ops,
                                          const double2 *__restrict__ mats, const double2 *lds_rt,
                                          const Ctx &c)
{
    const uint32_t ob = uni(H->op_begin), oe = uni(H->op_end);
    double2 b[16];
    for (uint32_t oi = ob; oi < oe; oi += 2) {
        apply_op(a, b, ops + oi, mats, lds_rt, c);
        if (oi + 1 < oe) {
            apply_op(b, a, ops + oi + 1, mats, lds_rt, c);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) a[e] = b[e];
        }
    }
}

// One HBM pass.  Persistent: workgroup b handles tiles b, b + G, b + 2G, ...
// and issues the loads of its next tile before working on the current one,
// so HBM traffic overlaps the FP64 work and the LDS exchanges.  Address
// parts that depend only on the thread are computed once; the tile and
// register-slot parts are workgroup-uniform (scalar unit).
template <bool PHANTOM>
__global__ void __launch_bounds__(1 << (kMaxTileBits - 4))
k_pass(const double2 *__restrict__ amps_in, double2 *__restrict__ amps_out, const KPass *__restrict__ passes,
       const KPhase *__restrict__ phases, const KOp *__restrict__ ops,
       const double2 *__restrict__ mats, uint32_t pass_idx)
{
    extern __shared__ double2 lds[];
    const KPass *P = passes + pass_idx;
    const uint32_t L = uni(P->L);
    const uint32_t nthr = L - 4;
    const uint32_t ngb = uni(P->n_group_bits);
    const bool xcd = uni(P->xcd_swizzle) != 0;
    const uint32_t n_tiles = (uint32_t)P->n_tiles;     // < 2^28
    const uint32_t tid = threadIdx.x;
    const uint32_t wave_base = uni(tid & ~63u);
    const uint32_t pb = uni(P->phase_begin), pe = uni(P->phase_end);
    const KPhase *H0 = phases + pb, *HL = phases + pe - 1;
    const bool multi_phase = pe - pb > 1;

    // stage the pass's runtime-diagonal factor tables in LDS after the tile
    const uint32_t rt_count = uni(P->rt_count);
    double2 *lds_rt = lds + ((pe - pb > 1) ? (1u << L) : 0u);
    if (rt_count) {
        const double2 *src = mats + uni(P->rt_mat);
        for (uint32_t i = tid; i < rt_count; i += blockDim.x) lds_rt[i] = src[i];
        __syncthreads();
    }

    // thread parts of the load (first phase) and store (last phase) addresses
    uint32_t tl0, tlL;
    uint32_t tg0, tgL;
    thread_bits(H0, tid, nthr, tl0, tg0);
    thread_bits(HL, tid, nthr, tlL, tgL);
    // (amps_in and amps_out are one buffer unless the pass changes the
    // layout; even then no load reads an address stored in the same launch:
    // tiles are disjoint and a tile loads before it stores)
    const double2 *ld_lane = amps_in + tg0;
    double2 *st_lane = amps_out + tgL;
    // Hermitian mode: thread parts of the mirrored store (the transpose of
    // tgL) and of the transposed load (of tg0); the previous pass's group
    // pair (i, j) of a loaded amplitude splits into a per-thread part and
    // per-register-bit parts (the bits come from disjoint sources)
    const uint32_t herm = uni(P->herm);
    uint32_t tgM = 0, tg0M = 0;
    HalfIn hin{};
    if (herm) {
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)kMaxThreadBits; ++i) {
            tgM |= ((tid >> i) & 1u) << (uni(HL->thr_mpos[i]) & 31u);
            tg0M |= ((tid >> i) & 1u) << (uni(H0->thr_mpos[i]) & 31u);
        }
        if (herm & kHermHalfIn) hin = half_in(P, tg0);
    }
    double2 *st_mirror = amps_out + tgM;
    const double2 *ld_mirror = amps_in + tg0M;

    uint32_t t = blockIdx.x;
    double2 nxt[16];
    HermTile ht_nxt{0u, 0u, 0u, 0u, false, true};     // Hermitian mode: the prefetched tile
    if (t < n_tiles) {
        if (herm) {
            ht_nxt = herm_tile(P, t, ngb, herm);
            load_herm(nxt, ld_lane, ld_mirror, ht_nxt, P, H0, herm, hin);
        } else {
            const uint32_t gb = group_base(P, t, ngb, xcd);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t u = gb | slot_g(H0, e);
                nxt[e] = (PHANTOM && ((u | tg0) >> kPhantomPos)) ? make_double2(0.0, 0.0) : ld_lane[u];
            }
        }
    }

    // Software pipeline, per tile t: wait for t's prefetched data, issue
    // the stores of the previous tile, issue the prefetch of the next tile,
    // then compute t.  The wait comes before the stores because the memory
    // counter retires in order: waiting for loads issued before fresh stores
    // would wait for those stores too.
    double2 a[16];
    uint32_t gb_prev = 0, gbm_prev = 0;
    bool have_prev = false, mirror_prev = false, valid_prev = true;
    for (; t < n_tiles; t += gridDim.x) {
        // vmcnt(0), other counters untouched (gfx9 encoding): the tile's
        // prefetch and the stores issued a whole tile ago; also keeps the
        // compiler from hoisting the stores below above this point
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // One barrier per tile serves two orderings:
        // * within a phase each thread writes back to the LDS slots it read,
        //   so phases need a barrier only between the writes and the next
        //   reads; but the first writes of this tile land in slots that other
        //   threads read in the previous tile's last phase;
        // * Hermitian mode with half storage: in a tile with i = j the waves
        //   load each other's amplitudes (through the transpose), so no wave
        //   may store the previous tile (below) before every wave has loaded
        //   it.
        if ((herm & kHermHalfIn) || multi_phase) __syncthreads();
        double2 cur[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) cur[e] = nxt[e];
        if (have_prev && valid_prev) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t u = gb_prev | slot_g(HL, e);
                if (!(PHANTOM && ((u | tgL) >> kPhantomPos))) st_lane[u] = a[e];
            }
            if (mirror_prev) store_mirror(st_mirror, gbm_prev, HL, a);
        }
        const HermTile ht = ht_nxt;              // the tile prefetched last iteration
        const uint32_t gb = herm ? ht.gb : group_base(P, t, ngb, xcd);
        {
            // prefetch the next tile (the last iteration re-reads its own
            // tile, which keeps the loads unconditional)
            const uint32_t t2 = (t + gridDim.x < n_tiles) ? t + gridDim.x : t;
            if (herm) {
                if (t2 != t) ht_nxt = herm_tile(P, t2, ngb, herm);
                load_herm(nxt, ld_lane, ld_mirror, ht_nxt, P, H0, herm, hin);
            } else {
                const uint32_t gb2 = group_base(P, t2, ngb, xcd);
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const uint32_t u = gb2 | slot_g(H0, e);
                    nxt[e] = (PHANTOM && ((u | tg0) >> kPhantomPos)) ? make_double2(0.0, 0.0) : ld_lane[u];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) a[e] = cur[e];

        for (uint32_t ph = pb; ph < pe; ++ph) {
            const KPhase *H = phases + ph;
            Ctx c;
            c.gb = gb;
#pragma unroll
            for (int b = 0; b < 4; ++b) c.rl[b] = 1u << uni(H->reg_local[b]);
            // the thread id is rebuilt from the lane id (mbcnt) and the
            // wave's uniform base rather than kept live in a register
            c.tl = (ph == pb) ? tl0 : (ph == pe - 1) ? tlL : thread_local_bits(H, lane_tid(wave_base), nthr);
            // LDS byte address of slot e: swizzle is xor-linear, so it splits
            // into a per-thread part and a uniform per-slot part
            const uint32_t lds_thr = swz(c.tl) << 4;
            if (ph != pb) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    a[e] = *reinterpret_cast<const double2 *>(
                        reinterpret_cast<const char *>(lds) + (lds_thr ^ uni(H->lds_slot[e])));
            }
            apply_ops(a, H, ops, mats, lds_rt, c);
            if (ph + 1 < pe) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    *reinterpret_cast<double2 *>(reinterpret_cast<char *>(lds) +
                                                 (lds_thr ^ uni(H->lds_slot[e]))) = a[e];
                __syncthreads();
            }
        }
        // the stores stay outside the phase loop: a loop holding global
        // stores but no loads makes the compiler wait for every outstanding
        // load (the prefetch) before entering it
        gb_prev = herm ? ht.gbs : gb;
        gbm_prev = ht.gbms;
        mirror_prev = ht.mirror && ht.valid && (herm & kHermMirror);
        valid_prev = ht.valid;
        have_prev = true;
    }
    if (have_prev && valid_prev) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t u = gb_prev | slot_g(HL, e);
            if (!(PHANTOM && ((u | tgL) >> kPhantomPos))) st_lane[u] = a[e];
        }
        if (mirror_prev) store_mirror(st_mirror, gbm_prev, HL, a);
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

// Fixed-order sums of the diagonal partials (layout [block][2 + n]) written
// to separate outputs: trace (re, im) to tr, <Z_i> to z (either may be null).
__global__ void __launch_bounds__(kThreads)
k_finish_diag(const double *__restrict__ partials, int nb, int n, double *__restrict__ tr,
              double *__restrict__ z)
{
    __shared__ double smem[4];
    const int nv = 2 + n;
    for (int k = 0; k < nv; ++k) {
        if ((k < 2 && !tr) || (k >= 2 && !z)) continue;
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nb; b += blockDim.x) v[0] += partials[(size_t)b * nv + k];
        block_sum<1>(v, smem);
        if (threadIdx.x == 0) {
            if (k < 2) tr[k] = v[0];
            else z[k - 2] = v[0];
        }
        __syncthreads();
    }
}

// Fixed-order sum of the Pauli partials (layout [block][2]) times i^ny.
__global__ void __launch_bounds__(kThreads)
k_finish_pauli(const double *__restrict__ partials, int nb, int ny, double *__restrict__ out)
{
    __shared__ double smem[8];
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        v[0] += partials[(size_t)b * 2];
        v[1] += partials[(size_t)b * 2 + 1];
    }
    block_sum<2>(v, smem);
    if (threadIdx.x == 0) {
        double a = v[0], c = v[1];
        for (int k = 0; k < (ny & 3); ++k) {
            const double t = a;
            a = -c;
            c = t;
        }
        out[0] = a;
        out[1] = c;
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

// ------------------------------------------------------------- batched --
// The register phases of one tile of the batched kernel (data in a).
__device__ __forceinline__ void batch_phases(double2 (&a)[16], const KPhase *__restrict__ phases,
                                             const KOp *__restrict__ ops, const double2 *__restrict__ mats,
                                             double2 *lds, const double2 *lds_rt, uint32_t pb, uint32_t pe,
                                             uint32_t gb, uint32_t tl0, uint32_t tlL, uint32_t wave_base,
                                             uint32_t nthr, bool active)
{
    for (uint32_t ph = pb; ph < pe; ++ph) {
        const KPhase *H = phases + ph;
        Ctx c;
        c.gb = gb;
#pragma unroll
        for (int b = 0; b < 4; ++b) c.rl[b] = 1u << uni(H->reg_local[b]);
        c.tl = (ph == pb) ? tl0 : (ph == pe - 1) ? tlL
             : thread_local_bits(H, active ? lane_tid(wave_base) : 0u, nthr);
        const uint32_t lds_thr = swz(c.tl) << 4;
        // a thread writes back to the slots it read, so only the writes
        // need a barrier before the next phase's reads (the first writes of
        // a tile are ordered after the previous tile's reads by batch_pass)
        if (ph != pb && active) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                a[e] = *reinterpret_cast<const double2 *>(
                    reinterpret_cast<const char *>(lds) + (lds_thr ^ uni(H->lds_slot[e])));
        }
        if (active) apply_ops(a, H, ops, mats, lds_rt, c);
        if (ph + 1 < pe) {
            if (active) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    *reinterpret_cast<double2 *>(reinterpret_cast<char *>(lds) +
                                                 (lds_thr ^ uni(H->lds_slot[e]))) = a[e];
            }
            __syncthreads();
        }
    }
}

// All tiles of one pass of one instance, software-pipelined: while tile t is
// computed in one register buffer, tile t+1 is loaded into the other (the
// loop is unrolled by two so that no loaded buffer is copied, which would
// wait for the load).  Per step: wait for the loads, issue the stores of the
// previous tile from the other buffer, prefetch into it, compute.  Loads are
// unconditional (inactive threads read thread 0's addresses and ignore the
// data); stores are not.
__device__ __forceinline__ void batch_pass(double2 *__restrict__ amps, const KPass *__restrict__ P,
                                           const KPhase *__restrict__ phases,
                                           const KOp *__restrict__ ops,
                                           const double2 *__restrict__ mats, double2 *lds,
                                           const double2 *lds_rt, uint32_t tid, uint32_t nthr, bool active)
{
    const uint32_t pb = uni(P->phase_begin), pe = uni(P->phase_end);
    const KPhase *H0 = phases + pb, *HL = phases + pe - 1;
    const uint32_t ngb = uni(P->n_group_bits);
    const uint32_t n_tiles = (uint32_t)P->n_tiles;
    const uint32_t L = uni(P->L);
    uint32_t tl0, tlL;
    uint32_t tg0, tgL;
    const uint32_t ttid = active ? tid : 0u;
    thread_bits(H0, ttid, nthr, tl0, tg0);
    thread_bits(HL, ttid, nthr, tlL, tgL);
    const double2 *ld_lane = amps + tg0;
    double2 *st_lane = amps + tgL;
    const uint32_t wave_base = uni(tid & ~63u);
    // Hermitian mode, as in k_pass: tile pairs i <= j, the previous pass's
    // stored half read directly or through the transpose, mirror images in
    // the instance's last pass
    const uint32_t herm = uni(P->herm);
    uint32_t tgM = 0, tg0M = 0;
    HalfIn hin{};
    if (herm) {
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)kMaxThreadBits; ++i) {
            tgM |= ((ttid >> i) & 1u) << (uni(HL->thr_mpos[i]) & 31u);
            tg0M |= ((ttid >> i) & 1u) << (uni(H0->thr_mpos[i]) & 31u);
        }
        if (herm & kHermHalfIn) hin = half_in(P, tg0);
    }
    double2 *st_mirror = amps + tgM;
    const double2 *ld_mirror = amps + tg0M;
    auto tile_at = [&](uint32_t t) {
        if (herm) return herm_tile(P, t, ngb, herm);
        const uint32_t gb = group_base(P, t, ngb, false);
        HermTile h{gb, 0u, gb, 0u, false, true};
        return h;
    };
    auto load = [&](double2 (&v)[16], const HermTile &h) {
        if (herm) {
            load_herm(v, ld_lane, ld_mirror, h, P, H0, herm, hin);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = ld_lane[h.gb | slot_g(H0, e)];
        }
    };
    auto store = [&](const double2 (&v)[16], const HermTile &h) {
        if (!active || !h.valid) return;
#pragma unroll
        for (int e = 0; e < 16; ++e) st_lane[h.gbs | slot_g(HL, e)] = v[e];
        if (h.mirror && (herm & kHermMirror)) store_mirror(st_mirror, h.gbms, HL, v);
    };
    // one barrier per tile: a tile with i = j is read through the transpose
    // by other waves than the ones that store it, so every wave's loads come
    // before any store; and the tile's first LDS writes come after the
    // previous tile's last LDS reads
    const bool half_in_sync = (herm & kHermHalfIn) != 0 || pe - pb > 1;
    double2 A[16], B[16];
    load(A, tile_at(0));
    for (uint32_t t = 0; t < n_tiles; t += 2) {
        // tile t in A; the previous tile's results are in B
        __builtin_amdgcn_s_waitcnt(0x0F70);          // vmcnt(0) only (gfx9 encoding)
        if (half_in_sync) __syncthreads();
        const HermTile h0 = tile_at(t);
        if (t > 0) store(B, tile_at(t - 1));
        load(B, tile_at((t + 1 < n_tiles) ? t + 1 : t));
        batch_phases(A, phases, ops, mats, lds, lds_rt, pb, pe, h0.gb, tl0, tlL, wave_base, nthr, active);
        if (t + 1 >= n_tiles) break;
        // tile t + 1 in B; tile t's results in A
        __builtin_amdgcn_s_waitcnt(0x0F70);
        if (half_in_sync) __syncthreads();
        const HermTile h1 = tile_at(t + 1);
        store(A, h0);
        load(A, tile_at((t + 2 < n_tiles) ? t + 2 : t + 1));
        batch_phases(B, phases, ops, mats, lds, lds_rt, pb, pe, h1.gb, tl0, tlL, wave_base, nthr, active);
    }
    // the last tile's results: in A when n_tiles is odd, else in B
    if (n_tiles > 0) {
        const HermTile hl = tile_at(n_tiles - 1);
        if (n_tiles & 1u) store(A, hl);
        else store(B, hl);
    }
}

// Global stores of this workgroup become visible to its own later loads
// (the vector L1 is not coherent with writes of other waves).
__device__ __forceinline__ void wg_global_sync()
{
    __threadfence();
    __syncthreads();
    __threadfence();
}

constexpr int kBatchThreads = 256;
constexpr int kBatchTileBits = 12;

// Persistent batched run: each workgroup takes the next instance from a
// largest-first queue, sets it to |0..0><0..0|, applies all of its passes
// (every tile of a pass by this workgroup, then a workgroup-wide sync), and
// writes <Z_i>, i < n, of the final state to its output slots.
__global__ void __launch_bounds__(kBatchThreads)
k_batch(double2 *__restrict__ arena, const BatchItem *__restrict__ items, uint32_t n_items,
        uint32_t *__restrict__ counter, const KPass *__restrict__ passes,
        const KPhase *__restrict__ phases, const KOp *__restrict__ ops,
        const double2 *__restrict__ mats, double *__restrict__ out)
{
    extern __shared__ double2 lds[];
    __shared__ uint32_t s_item;
    __shared__ double s_red[VQD_MAX_QUBITS * 4];
    double2 *lds_rt = lds + (1u << kBatchTileBits);
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem *B = items + it;
        const uint32_t n = uni(B->n);
        const double2 *M = mats + B->mat_base;     // this instance's coefficients
        double2 *amps = arena + B->arena_off;
        const uint64_t count = 1ull << (2 * n);
        for (uint64_t i = tid; i < count; i += blockDim.x) amps[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
        wg_global_sync();
        const uint32_t qb = uni(B->pass_begin), qe = uni(B->pass_end);
        for (uint32_t p = qb; p < qe; ++p) {
            const KPass *P = passes + p;
            const uint32_t L = uni(P->L), nthr = L - 4;
            const bool active = tid < (1u << nthr);
            const uint32_t rt_count = uni(P->rt_count);
            if (rt_count) {
                const double2 *src = M + uni(P->rt_mat);
                for (uint32_t i = tid; i < rt_count; i += blockDim.x) lds_rt[i] = src[i];
                __syncthreads();
            }
            batch_pass(amps, P, phases, ops, M, lds, lds_rt, tid, nthr, active);
            wg_global_sync();
        }
        // <Z_q> = sum_r (-1)^{r_q} Re rho[r][r]
        double z[VQD_MAX_QUBITS];
#pragma unroll
        for (int q = 0; q < VQD_MAX_QUBITS; ++q) z[q] = 0.0;
        const uint64_t D = 1ull << n;
        for (uint64_t r = tid; r < D; r += blockDim.x) {
            const double pr = amps[r * (D + 1)].x;
#pragma unroll
            for (int q = 0; q < VQD_MAX_QUBITS; ++q)
                if ((uint32_t)q < n) z[q] += ((r >> q) & 1u) ? -pr : pr;
        }
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int q = 0; q < VQD_MAX_QUBITS; ++q) {
            double v = z[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) s_red[q * 4 + wv] = v;
        }
        __syncthreads();
        if (tid < n) {
            const double v = (s_red[tid * 4] + s_red[tid * 4 + 1]) + (s_red[tid * 4 + 2] + s_red[tid * 4 + 3]);
            out[B->out_off + tid] = v;
        }
        __syncthreads();
    }
}

__global__ void k_reset(uint32_t *counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

}  // namespace

// ------------------------------------------------------------- launches --
int launch_pass(double2 *amps_in, double2 *amps_out, const DevProgram &dev, const KPass &pass,
                uint32_t pass_idx, hipStream_t stream)
{
    const uint32_t threads = 1u << (pass.L - 4);
    const size_t lds = ((pass.phase_end - pass.phase_begin > 1) ? (size_t(16) << pass.L) : 0) +
                       size_t(16) * pass.rt_count;
    if (lds > 160 * 1024) return fail(VQD_E_SIZE, "pass needs more LDS than a workgroup has");
    static bool attr_set = false;
    static int n_cu = 0;
    const void *kfn = pass.phantom ? (const void *)k_pass<true> : (const void *)k_pass<false>;
    if (!attr_set) {
        VQD_HIP(hipFuncSetAttribute((const void *)k_pass<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024));
        VQD_HIP(hipFuncSetAttribute((const void *)k_pass<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024));
        int dev_id = 0;
        VQD_HIP(hipGetDevice(&dev_id));
        VQD_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id));
        attr_set = true;
    }
    // persistent grid: as many workgroups as fit on the device at once
    int per_cu = 0;
    VQD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, (int)threads, lds));
    if (per_cu < 1) per_cu = 1;
    uint64_t grid = (uint64_t)per_cu * (uint64_t)n_cu;
    grid -= grid % 64;               // keeps the XCD tile mapping a bijection
    if (grid == 0) grid = 64;
    if (grid > pass.n_tiles) grid = pass.n_tiles;
    if (pass.phantom)
        hipLaunchKernelGGL(k_pass<true>, dim3((uint32_t)grid), dim3(threads), lds, stream, amps_in, amps_out,
                           dev.passes, dev.phases, dev.ops, dev.mats, pass_idx);
    else
        hipLaunchKernelGGL(k_pass<false>, dim3((uint32_t)grid), dim3(threads), lds, stream, amps_in, amps_out,
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

// ------------------------------------------------- device-output read-outs --
// The same kernels as the synchronous read-outs, writing into caller device
// memory; the partials go to a scratch that is allocated once per handle
// (never inside these calls), so that the calls can be captured in a graph.
size_t readout_scratch_doubles(int n)
{
    const uint64_t D = 1ull << n;
    const size_t diag = (size_t)256 * (2 + n) + D;      // partials, then the probabilities (<ZZ>)
    return std::max<size_t>(diag, kRedBlocks) + 8;
}

static int check_readout_scratch(const ReduceScratch &s, int n)
{
    if (!s.dev || s.cap < readout_scratch_doubles(n))
        return fail(VQD_E_NOMEM, "no device read-out scratch (the handle was wrapped without a GPU)");
    return VQD_OK;
}

int reduce_purity_dev(const double2 *amps, int n, const ReduceScratch &s, hipStream_t st, double *out)
{
    if (int rc = check_readout_scratch(s, n)) return rc;
    const uint64_t count = 1ull << (2 * n);
    uint64_t blocks = (count + kThreads - 1) / kThreads;
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL(k_purity, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, count, s.dev);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, st, s.dev, (int)blocks, 1, out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int reduce_diag_dev(const double2 *amps, int n, const ReduceScratch &s, hipStream_t st, double *tr, double *z,
                    double *probs)
{
    if (int rc = check_readout_scratch(s, n)) return rc;
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(k_diag, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n, probs, s.dev);
    VQD_HIP(hipGetLastError());
    if (tr || z) {
        hipLaunchKernelGGL(k_finish_diag, dim3(1), dim3(kThreads), 0, st, s.dev, (int)blocks, n, tr, z);
        VQD_HIP(hipGetLastError());
    }
    return VQD_OK;
}

int reduce_zz_dev(const double2 *amps, int n, const int *pairs, int npairs, const ReduceScratch &s,
                  hipStream_t st, double *out)
{
    if (int rc = check_readout_scratch(s, n)) return rc;
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    double *probs = s.dev + (size_t)256 * (2 + n);
    hipLaunchKernelGGL(k_diag, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n, probs, s.dev);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_zz, dim3(npairs), dim3(kThreads), 0, st, probs, n, reinterpret_cast<const int2 *>(pairs),
                       out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int reduce_pauli_dev(const double2 *amps, int n, uint64_t xmask, uint64_t zmask, int ny, const ReduceScratch &s,
                     hipStream_t st, double *out)
{
    if (int rc = check_readout_scratch(s, n)) return rc;
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    hipLaunchKernelGGL(k_pauli, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n, xmask, zmask, s.dev);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_pauli, dim3(1), dim3(kThreads), 0, st, s.dev, (int)blocks, ny, out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

// ----------------------------------------------- read-out without allocation --
// The partials of vqd_calc_expec_z_noalloc: one file-scope device array,
// sized for the largest state (256 blocks of 2 + VQD_MAX_QUBITS sums).  Each
// GPU the library runs on holds its own copy until the process ends.  In host
// code its name is not a device address; hipGetSymbolAddress gives each
// device's copy, kept in noalloc_scratch_ptr[device].
constexpr size_t kNoAllocScratch = (size_t)256 * (2 + VQD_MAX_QUBITS);
static __device__ __align__(256) double scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mutex;
static double *g_noalloc_ptr[kMaxDevices];

static int noalloc_scratch_ptr(double **out)
{
    int dev = 0;
    VQD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(VQD_E_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        // once per device, with that device current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e,
                                                   "hipGetSymbolAddress(scratch)");
        g_noalloc_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_noalloc_ptr[dev];
    return VQD_OK;
}

int expec_z_noalloc(const double2 *amps, int n, hipStream_t st, double *out)
{
    double *sc = nullptr;
    if (int rc = noalloc_scratch_ptr(&sc)) return rc;
    const uint64_t D = 1ull << n;
    uint64_t blocks = (D + kThreads - 1) / kThreads;
    if (blocks > 256) blocks = 256;
    if (blocks * (2 + (uint64_t)n) > kNoAllocScratch) return fail(VQD_E_SIZE, "state too large for the static scratch");
    // every block writes its own partials before k_finish_diag reads them,
    // so nothing left from an earlier call needs clearing
    hipLaunchKernelGGL(k_diag, dim3((uint32_t)blocks), dim3(kThreads), 0, st, amps, n, nullptr, sc);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_diag, dim3(1), dim3(kThreads), 0, st, sc, (int)blocks, n, nullptr, out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

int launch_batch(double2 *arena, const BatchDev &bd, double *out, hipStream_t stream)
{
    static bool attr = false;
    if (!attr) {
        // dynamic LDS plus the kernel's static queue and reduction slots
        VQD_HIP(hipFuncSetAttribute((const void *)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    159 * 1024));
        attr = true;
    }
    const size_t lds = (size_t(16) << kBatchTileBits) + size_t(16) * bd.max_rt;
    if (lds + 1024 > 160 * 1024) return fail(VQD_E_SIZE, "batched pass needs more LDS than a workgroup has");
    int per_cu = 0, n_cu = 0, dev_id = 0;
    VQD_HIP(hipGetDevice(&dev_id));
    VQD_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id));
    VQD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batch, kBatchThreads, lds));
    if (per_cu < 1) per_cu = 1;
    uint32_t grid = (uint32_t)per_cu * (uint32_t)n_cu;
    if (grid > bd.n_items) grid = bd.n_items;
    if (grid == 0) return VQD_OK;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, bd.counter);
    VQD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBatchThreads), lds, stream, arena, bd.items, bd.n_items,
                       bd.counter, bd.prog.passes, bd.prog.phases, bd.prog.ops, bd.prog.mats, out);
    VQD_HIP(hipGetLastError());
    return VQD_OK;
}

}  // namespace vqd
