// Host planner: turns an ordered op list into HBM passes, register phases and
// kernel ops.
//
// Dependencies.  Two ops must keep their order if they share a qubit, unless
// both are diagonal (element-wise products commute).
//
// Passes.  A pass owns a qubit set Q whose row and column bits, plus the
// lowest `min_contig_bits` vector bits, fit in the tile (<= tile_bits bits).
// Non-diagonal ops may join the pass only if their qubits lie in Q;
// diagonal ops may join wherever their dependencies allow, because their
// factor depends only on an amplitude's own index.  Q is grown greedily,
// each step adding the blocked op's qubits that let the most ops join.
// Hermitian plans with relabelled layouts replace the forced low qubits by
// one qubit shared with the previous tile (see plan_program_mode).
//
// Phases.  Inside a pass, ops are grouped into register phases of at most
// two qubits (4 register bits: row and column bit of each).  Ops of a phase
// are moved into the phase's 16-slot space, where runs that act on
// overlapping bits are multiplied into one block when that costs fewer FMAs
// (the product of superoperators is exact; this is the paper's own channel
// composition, eq. stderr, generalised).  Each resulting block is encoded in
// its cheapest form: a matrix on 2 or 4 register bits with its zero and real
// entries flagged, or element-wise factors.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "vqd_internal.h"

namespace vqd {

namespace {

using Mat16 = std::array<cd, 256>;

uint32_t qmask(const LOp &op)
{
    uint32_t m = 0;
    for (int j = 0; j < op.k; ++j) m |= 1u << op.q[j];
    return m;
}

int popc(uint32_t x) { return __builtin_popcount(x); }

// Global vector-bit positions of the pass tile for qubit set Q.
std::vector<int> tile_bits_for(uint32_t Q, int n, int contig)
{
    std::vector<int> b;
    for (int i = 0; i < contig && i < 2 * n; ++i) b.push_back(i);
    for (int q = 0; q < n; ++q)
        if (Q >> q & 1) {
            b.push_back(q);
            b.push_back(q + n);
        }
    std::sort(b.begin(), b.end());
    b.erase(std::unique(b.begin(), b.end()), b.end());
    return b;
}

// Does the op map every Hermitian matrix to a Hermitian one?  Under the
// transpose of the row and column bits (local index a -> mu(a)) such an op
// satisfies S[mu(a)][mu(b)] = conj(S[a][b]); a unitary applied as U on rows
// and conj(U) on columns always does.
bool preserves_hermiticity(const LOp &op)
{
    if (op.wide_unitary) return true;
    const int k = op.k, D = 1 << (2 * k), lo = (1 << k) - 1;
    auto mu = [&](int a) { return (a >> k) | ((a & lo) << k); };
    double scale = 0.0;
    const std::vector<cd> &v = op.diag ? op.D : op.S;
    for (const cd &x : v) scale = std::max(scale, std::abs(x));
    const double tol = 1e-13 * std::max(1.0, scale);
    if (op.diag) {
        for (int a = 0; a < D; ++a)
            if (std::abs(op.D[mu(a)] - std::conj(op.D[a])) > tol) return false;
        return true;
    }
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
            if (std::abs(op.S[size_t(mu(a)) * D + mu(b)] - std::conj(op.S[size_t(a) * D + b])) > tol) return false;
    return true;
}

struct SimResult {
    std::vector<int> taken;
    std::vector<uint32_t> cands;   // qubit sets of blocked non-diagonal ops
};

// Which ops (from `first`, not yet applied) can join a pass on qubit set Q.
void simulate(const std::vector<LOp> &ops, const std::vector<uint32_t> &qm,
              const std::vector<char> &applied, size_t first, uint32_t Q, int n,
              int max_take, SimResult &res, bool want_cands)
{
    res.taken.clear();
    res.cands.clear();
    const uint32_t all = (n >= 32) ? 0xffffffffu : ((1u << n) - 1);
    uint32_t blk_any = 0, blk_nd = 0;
    for (size_t i = first; i < ops.size(); ++i) {
        if (applied[i]) continue;
        const LOp &op = ops[i];
        const uint32_t m = qm[i];
        bool take = false, cand = false;
        if (m & blk_any) {
        } else if (!op.diag && (m & blk_nd)) {
        } else if (op.diag) {
            take = true;
        } else if ((m & ~Q) == 0) {
            take = true;
        } else {
            cand = true;
        }
        if (take) {
            res.taken.push_back((int)i);
            if (max_take > 0 && (int)res.taken.size() >= max_take) break;
        } else {
            if (op.diag) blk_nd |= m;
            else blk_any |= m;
            if (cand && want_cands) {
                if (std::find(res.cands.begin(), res.cands.end(), m) == res.cands.end() &&
                    res.cands.size() < 32)
                    res.cands.push_back(m);
            }
            if (blk_any == all) break;
        }
    }
}

// ---- slot-space blocks --------------------------------------------------

struct Block {
    bool rt = false;            // runtime-indexed diagonal (KOP_DIAG_RT)
    Mat16 m{};                  // slot-space matrix (when !rt)
    uint32_t support = 0;       // register bits the block depends on
    bool diag = false;
    int op_index = -1;          // for rt blocks
    std::vector<int> src;       // logical ops multiplied in, application order
    int wide_half = -1;         // wide unitary row (0) or column (1) half
};

bool is_zero(cd x) { return x.real() == 0.0 && x.imag() == 0.0; }

// Does m act as identity-extended on the complement of `mask`?  If so,
// extract the dim x dim matrix on `mask` (bits in ascending order).
bool restrict_to(const Mat16 &m, int mask, std::vector<cd> &sub)
{
    const int rest = (~mask) & 15;
    int nb = popc((uint32_t)mask), dim = 1 << nb;
    auto dep = [](int v, int msk) {
        int out = 0, k = 0;
        for (int b = 0; b < 4; ++b)
            if (msk >> b & 1) {
                if (v >> k & 1) out |= 1 << b;
                ++k;
            }
        return out;
    };
    sub.assign(size_t(dim) * dim, cd(0));
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) sub[i * dim + j] = m[dep(i, mask) * 16 + dep(j, mask)];
    // verify: every entry equals the block value when rest bits agree, else 0
    for (int so = 0; so < 16; ++so)
        for (int si = 0; si < 16; ++si) {
            cd v = m[so * 16 + si];
            if ((so & rest) != (si & rest)) {
                if (!is_zero(v)) return false;
                continue;
            }
            int i = 0, j = 0, k = 0;
            for (int b = 0; b < 4; ++b)
                if (mask >> b & 1) {
                    i |= ((so >> b) & 1) << k;
                    j |= ((si >> b) & 1) << k;
                    ++k;
                }
            if (v != sub[i * dim + j]) return false;
        }
    return true;
}

bool all_real(const std::vector<cd> &v)
{
    for (const cd &x : v)
        if (x.imag() != 0.0) return false;
    return true;
}

// Flip patterns of a register mask: flipping the row and the column bit of
// the same qubit together.  In slot space mask 5 holds one qubit on slot
// bits (0, 2), mask 10 one on (1, 3), mask 15 both.  Returned as local
// indices inside the mask (dep4 order).
std::vector<int> local_flips(int mask)
{
    if (mask == 5 || mask == 10) return {0, 3};
    if (mask == 15) return {0, 5, 10, 15};
    return {};
}

struct Encoded {
    uint32_t kind = KOP_MAT;
    int mask = 15;
    bool real = false;
    bool identity = false;
    std::vector<cd> data;   // kernel layout (see KOp)
    double cost = 0;        // FMAs per 16 slots
};

// Pack coefficients into the pool layout: complex as is, real ones two per entry.
std::vector<cd> pack(const std::vector<cd> &c, bool real)
{
    if (!real) return c;
    std::vector<cd> o((c.size() + 1) / 2);
    for (size_t i = 0; i < c.size(); ++i) {
        if (i & 1) o[i / 2].imag(c[i].real());
        else o[i / 2].real(c[i].real());
    }
    return o;
}

// Pauli transfer form of a map on two register bits (KOP_PTM).  sub is the
// 4x4 matrix (row-major, output index first) on the local index u + 2v of the
// block entry B[u][v].  R_PQ = Tr(P S(Q)) / 2 over P, Q in (I, X, Y, Z) is
// real exactly when S takes Hermitian blocks to Hermitian blocks, and its row
// I is (1, 0, 0, 0) exactly when S keeps the trace.  In floating point both
// hold up to the rounding of the planner's products: accepted to within
// kPtmTol.  rows gets the rows X, Y, Z of R / 2 (row-major, columns I, X, Y,
// Z); false when either property fails.
constexpr double kPtmTol = 1e-14;

bool ptm_of(const std::vector<cd> &sub, std::vector<double> &rows)
{
    const cd I1(0.0, 1.0);
    // the Pauli matrices as local vectors p_l = P[u][v], l = u + 2v
    const cd pv[4][4] = {{1.0, 0.0, 0.0, 1.0}, {0.0, 1.0, 1.0, 0.0}, {0.0, I1, -I1, 0.0}, {1.0, 0.0, 0.0, -1.0}};
    double R[4][4];
    for (int q = 0; q < 4; ++q) {
        cd sq[4];
        for (int i = 0; i < 4; ++i) {
            sq[i] = 0.0;
            for (int j = 0; j < 4; ++j) sq[i] += sub[i * 4 + j] * pv[q][j];
        }
        for (int p = 0; p < 4; ++p) {
            cd t = 0.0;    // Tr(P B) = sum_l conj(p_l) b_l for Hermitian P
            for (int l = 0; l < 4; ++l) t += std::conj(pv[p][l]) * sq[l];
            t *= 0.5;
            if (std::abs(t.imag()) > kPtmTol * std::max(1.0, std::abs(t.real()))) return false;
            R[p][q] = t.real();
        }
    }
    if (std::abs(R[0][0] - 1.0) > kPtmTol || std::abs(R[0][1]) > kPtmTol || std::abs(R[0][2]) > kPtmTol ||
        std::abs(R[0][3]) > kPtmTol)
        return false;
    rows.clear();
    for (int p = 1; p < 4; ++p)
        for (int q = 0; q < 4; ++q) rows.push_back(0.5 * R[p][q]);
    return true;
}

// FP64 work of a KOP_PTM per 16 slots in FMA units (an add or a multiply
// counts half): per group of 4 slots, 8 adds into the Pauli basis, 3 rows of
// 4 real coefficients times a complex vector (6 multiplies, 18 FMAs), then 4
// FMAs and 4 adds back.
constexpr double kPtmCost = 4 * 31.0;

// Cheapest branch-free kernel form of a slot-space matrix.
Encoded encode(const Mat16 &m)
{
    Encoded best;
    best.cost = 1e30;
    bool diag = true, ident = true;
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j) {
            const cd v = m[i * 16 + j];
            if (i != j && !is_zero(v)) diag = false;
            if (v != (i == j ? cd(1) : cd(0))) ident = false;
        }
    if (ident) {
        best.identity = true;
        best.cost = 0;
        return best;
    }
    if (diag) {
        std::vector<cd> f(16);
        for (int e = 0; e < 16; ++e) f[e] = m[e * 16 + e];
        best.kind = KOP_DIAG;
        best.real = all_real(f);
        best.data = pack(f, best.real);
        best.cost = 16.0 * (best.real ? 2 : 4);
        return best;
    }
    static const int masks[] = {5, 10, 15, 7};
    std::vector<cd> sub;
    for (int mask : masks) {
        if (!restrict_to(m, mask, sub)) continue;
        const int nb = popc((uint32_t)mask), dim = 1 << nb, groups = 16 >> nb;
        const bool real = all_real(sub);
        const double per = real ? 2.0 : 4.0;
        // dense, column-major
        const double dense = groups * dim * dim * per;
        if (dense < best.cost) {
            std::vector<cd> cm(size_t(dim) * dim);
            for (int j = 0; j < dim; ++j)
                for (int i = 0; i < dim; ++i) cm[j * dim + i] = sub[i * dim + j];
            best.kind = KOP_MAT;
            best.mask = mask;
            best.real = real;
            best.data = pack(cm, real);
            best.cost = dense;
        }
        // Pauli transfer form of a one-qubit map
        if (nb == 2 && kPtmCost < best.cost) {
            std::vector<double> rows;
            if (ptm_of(sub, rows)) {
                std::vector<cd> c(rows.begin(), rows.end());
                best.kind = KOP_PTM;
                best.mask = mask;
                best.real = true;
                best.data = pack(c, true);
                best.cost = kPtmCost;
            }
        }
        // flip pattern: nonzeros only where row and column bits flip together
        const std::vector<int> fl = local_flips(mask);
        if (fl.empty()) continue;
        bool ok = true;
        for (int i = 0; i < dim && ok; ++i)
            for (int j = 0; j < dim; ++j)
                if (!is_zero(sub[i * dim + j]) &&
                    std::find(fl.begin(), fl.end(), i ^ j) == fl.end()) { ok = false; break; }
        if (!ok) continue;
        const double xcost = groups * dim * (double)fl.size() * per;
        if (xcost < best.cost) {
            std::vector<cd> w(fl.size() * dim);
            for (size_t x = 0; x < fl.size(); ++x)
                for (int i = 0; i < dim; ++i) w[x * dim + i] = sub[i * dim + (i ^ fl[x])];
            best.kind = KOP_XOR;
            best.mask = mask;
            best.real = real;
            best.data = pack(w, real);
            best.cost = xcost;
        }
    }
    return best;
}

Mat16 mul(const Mat16 &B, const Mat16 &A)   // B * A (A applied first)
{
    Mat16 C{};
    for (int i = 0; i < 16; ++i)
        for (int k = 0; k < 16; ++k) {
            const cd b = B[i * 16 + k];
            if (is_zero(b)) continue;
            for (int j = 0; j < 16; ++j) C[i * 16 + j] += b * A[k * 16 + j];
        }
    return C;
}

// Embed a k<=2 op into slot space.  slot_of_gpos maps a global bit to its
// register bit (or -1).
Mat16 embed(const LOp &op, int n, const int *reg_gpos, uint32_t &support)
{
    const int k = op.k, nb = 2 * k, D = 1 << nb;
    int sbit[4];
    support = 0;
    for (int j = 0; j < nb; ++j) {
        const int g = (j < k) ? op.q[j] : op.q[j - k] + n;
        sbit[j] = -1;
        for (int b = 0; b < 4; ++b)
            if (reg_gpos[b] == g) sbit[j] = b;
        support |= 1u << sbit[j];
    }
    auto local = [&](int slot) {
        int l = 0;
        for (int j = 0; j < nb; ++j) l |= ((slot >> sbit[j]) & 1) << j;
        return l;
    };
    Mat16 m{};
    for (int so = 0; so < 16; ++so)
        for (int si = 0; si < 16; ++si) {
            if ((so & ~support) != (si & ~support)) continue;
            const int lo = local(so), li = local(si);
            cd v;
            if (op.diag) v = (lo == li) ? op.D[lo] : cd(0);
            else v = op.S[size_t(lo) * D + li];
            m[so * 16 + si] = v;
        }
    return m;
}


}  // namespace

void rt_table(uint32_t mode, int ubits, const std::vector<RtPart> &parts, const std::vector<LOp> &ops,
              std::vector<cd> &table)
{
    if (mode == RT_GENERIC) {            // one op, every index bit gathered in its own order
        table = ops[parts[0].src].D;
        return;
    }
    const int shift = (mode == RT_NONE) ? 0 : 2;
    table.assign(size_t(1) << (shift + ubits), cd(1));
    for (const RtPart &pt : parts) {
        const std::vector<cd> &D = ops[pt.src].D;
        for (int t = 0; t < (1 << ubits); ++t)
            for (int c = 0; c < (1 << shift); ++c) {
                int idx = 0;
                for (size_t k = 0; k < pt.rtj.size(); ++k) idx |= ((t >> pt.upos[k]) & 1) << pt.rtj[k];
                if (pt.mode != RT_NONE) idx |= ((c & 1) << pt.row_j) | (((c >> 1) & 1) << pt.col_j);
                table[size_t(c) + (size_t(t) << shift)] *= D[idx];
            }
    }
}

namespace {

// ---- relabelled layouts (PlanOpts::relayout) ------------------------------
// A layout phi gives each logical index bit b (row bit q = b < n, column bit
// q = b - n) its physical position phi[b].  The vectorised layout of the
// caller's buffer is the identity.  Between two passes of a relabelled plan
// the state is stored interleaved: qubit q in slot s(q) has its row bit at
// position 2 s(q) and its column bit at 2 s(q) + 1, so a tile whose qubits
// hold the lowest slots is one contiguous block.  Either way the transpose
// of a physical index exchanges the two bits of each qubit.
using Layout = std::vector<int>;

Layout vectorised(int n)
{
    Layout phi(2 * n);
    for (int b = 0; b < 2 * n; ++b) phi[b] = b;
    return phi;
}

Layout interleaved(int n, const std::vector<int> &order)    // order[s] = qubit in slot s
{
    Layout phi(2 * n);
    for (int s = 0; s < n; ++s) {
        phi[order[s]] = 2 * s;
        phi[order[s] + n] = 2 * s + 1;
    }
    return phi;
}

// Position of the transpose partner of physical position p under phi.
uint32_t mirror_under(const Layout &phi, int n, uint32_t p)
{
    for (int b = 0; b < 2 * n; ++b)
        if ((uint32_t)phi[b] == p) return (uint32_t)phi[b < n ? b + n : b - n];
    return p;
}

// Lane order of a phase that loads or stores HBM: the longest run of
// physical positions 0, 1, 2, ... among its thread bits, then the transpose
// partners of those (the mirrored stores and transposed loads), then the
// other thread bits in their order.
void coalesce_lanes(KPhase &H, uint32_t nthr, const Layout &phi, int n)
{
    auto slot_of = [&](uint32_t g) {
        for (uint32_t t = 0; t < nthr; ++t)
            if (H.thr_gpos[t] == g) return (int)t;
        return -1;
    };
    std::vector<uint32_t> want;
    for (uint32_t p = 0; slot_of(p) >= 0; ++p) want.push_back(p);
    const size_t run = want.size();
    for (size_t k = 0; k < run; ++k) {
        const uint32_t mp = mirror_under(phi, n, want[k]);
        if (slot_of(mp) >= 0 && std::find(want.begin(), want.end(), mp) == want.end()) want.push_back(mp);
    }
    std::vector<uint32_t> order;                    // thread entries in lane order
    for (uint32_t g : want) order.push_back((uint32_t)slot_of(g));
    for (uint32_t t = 0; t < nthr; ++t)
        if (std::find(want.begin(), want.end(), H.thr_gpos[t]) == want.end()) order.push_back(t);
    const KPhase old = H;       // the mirror table moves with its entries
    for (uint32_t t = 0; t < nthr; ++t) {
        H.thr_local[t] = old.thr_local[order[t]];
        H.thr_gpos[t] = old.thr_gpos[order[t]];
        H.thr_mpos[t] = old.thr_mpos[order[t]];
    }
}

// The phase's positions (logical so far) under phi, with their mirror table.
void place_phase(KPhase &H, uint32_t nthr, const Layout &phi, int n)
{
    for (int b = 0; b < kRegBits; ++b) {
        H.reg_gpos[b] = (uint32_t)phi[H.reg_gpos[b]];
        H.reg_mpos[b] = mirror_under(phi, n, H.reg_gpos[b]);
    }
    for (uint32_t t = 0; t < (uint32_t)kMaxThreadBits; ++t) {
        if (t < nthr) {
            H.thr_gpos[t] = (uint32_t)phi[H.thr_gpos[t]];
            H.thr_mpos[t] = mirror_under(phi, n, H.thr_gpos[t]);
        } else {
            H.thr_gpos[t] = H.thr_mpos[t] = 0;
        }
    }
}

// The passes of a Hermitian plan, built with logical bit positions, get a
// layout for the state between every two of them, and every position the
// kernel reads is rewritten for the layout it applies to: the group bits and
// the first phase for the layout the pass loads, out_gpos and the last phase
// for the one it stores, runtime-diagonal gathers for the loaded one (the
// kernel takes their group bits from the load base).
//
// The layout before pass b is interleaved with pass b's tile qubits in the
// lowest slots: the qubits pass b-1 also holds in its tile (and in no
// register of its storing or pass b's loading phase) first, pass b's other
// thread qubits next, its first phase's register qubits last, then the
// other qubits in their previous order.  Pass b then loads one contiguous
// block per tile, and pass b-1 stores runs of 4^c amplitudes, c the shared
// qubits in front.
//
// Constraints: the first pass loads and the last stores the vectorised
// layout; a single-phase pass keeps its layout (its one phase loads and
// stores); a pass that changes the layout stores into the other buffer, so
// the number of changes is made even by giving up the least useful one.
bool relabel_passes(int n, HostPlan &plan)
{
    const size_t K = plan.passes.size();
    if (K < 2) return true;
    const uint32_t full = (1u << n) - 1u;
    struct PInfo {
        uint32_t tile = 0, reg_first = 0, reg_last = 0;
        bool single = false;
    };
    std::vector<PInfo> info(K);
    auto reg_qubits = [&](const KPhase &H) {
        uint32_t m = 0;
        for (int b = 0; b < kRegBits; ++b)
            if (H.reg_gpos[b] < 2u * (uint32_t)n) m |= 1u << (H.reg_gpos[b] % (uint32_t)n);
        return m;
    };
    for (size_t p = 0; p < K; ++p) {
        const KPass &P = plan.passes[p];
        const uint32_t m = P.n_group_bits >> 1;
        uint32_t g = 0;
        for (uint32_t k = 0; k < m; ++k) g |= 1u << P.group_gpos[k];
        info[p].tile = full & ~g;
        info[p].reg_first = reg_qubits(plan.phases[P.phase_begin]);
        info[p].reg_last = reg_qubits(plan.phases[P.phase_end - 1]);
        info[p].single = P.phase_end - P.phase_begin == 1;
    }
    const Layout vec = vectorised(n);
    std::vector<Layout> lam(K + 1, vec);
    std::vector<int> width(K + 1, 0);
    std::vector<int> slot(n);                       // the previous boundary's slots
    for (int q = 0; q < n; ++q) slot[q] = q;
    for (size_t b = 1; b < K; ++b) {
        const uint32_t T = info[b].tile, R = info[b].reg_first;
        const uint32_t C = info[b - 1].tile & T & ~info[b - 1].reg_last & ~R;
        std::vector<int> groups[4];                 // C, T \ C \ R, R, the others
        for (int q = 0; q < n; ++q)
            groups[(C >> q & 1) ? 0 : !(T >> q & 1) ? 3 : (R >> q & 1) ? 2 : 1].push_back(q);
        std::vector<int> order;
        for (auto &gr : groups) {
            std::stable_sort(gr.begin(), gr.end(), [&](int x, int y) { return slot[x] < slot[y]; });
            order.insert(order.end(), gr.begin(), gr.end());
        }
        for (int s = 0; s < n; ++s) slot[order[s]] = s;
        lam[b] = interleaved(n, order);
        width[b] = __builtin_popcount(C);
    }
    // runs of single-phase passes share one layout; at the program's ends
    // it is the vectorised one
    for (size_t p = 0; p < K;) {
        if (!info[p].single) {
            ++p;
            continue;
        }
        size_t q = p;
        while (q + 1 < K && info[q + 1].single) ++q;
        const Layout keep = (p == 0 || q + 1 == K) ? vec : lam[p];
        for (size_t b = p; b <= q + 1; ++b) lam[b] = keep;
        p = q + 1;
    }
    auto changes = [&]() {
        size_t c = 0;
        for (size_t p = 0; p < K; ++p) c += lam[p] != lam[p + 1] ? 1 : 0;
        return c;
    };
    if (changes() % 2) {
        size_t best = 0;
        for (size_t b = 1; b < K; ++b) {
            if (info[b - 1].single || info[b].single || lam[b] == lam[b - 1]) continue;
            const Layout keep = lam[b];
            lam[b] = lam[b - 1];
            const bool even = changes() % 2 == 0;
            lam[b] = keep;
            if (even && (best == 0 || width[b] < width[best])) best = b;
        }
        if (best) lam[best] = lam[best - 1];
        else std::fill(lam.begin(), lam.end(), vec);
    }
    // whether every pass loads and stores with its lowest physical qubit (the
    // one whose row bit is position 0) outside the registers of the phase
    // doing it, so that its lanes start on a contiguous run
    bool io_ok = true;
    auto lowest = [&](const Layout &phi) {
        for (int q = 0; q < n; ++q)
            if (phi[q] == 0) return q;
        return 0;
    };
    for (size_t p = 0; p < K; ++p) {
        const uint32_t in_q = 1u << lowest(lam[p]), out_q = 1u << lowest(lam[p + 1]);
        io_ok = io_ok && (info[p].tile & in_q) && !(info[p].reg_first & in_q);
        io_ok = io_ok && (info[p].tile & out_q) && !(info[p].reg_last & out_q);
    }
    for (size_t p = 0; p < K; ++p) {
        KPass &P = plan.passes[p];
        const Layout &li = lam[p], &lo = lam[p + 1];
        P.swap_out = (li != lo) ? 1u : 0u;
        plan.alt_buffer = plan.alt_buffer || P.swap_out != 0;
        const uint32_t m = P.n_group_bits >> 1;
        std::vector<int> gq;
        for (uint32_t k = 0; k < m; ++k) gq.push_back((int)P.group_gpos[k]);
        std::stable_sort(gq.begin(), gq.end(), [&](int x, int y) { return li[x] < li[y]; });
        for (uint32_t k = 0; k < m; ++k) {
            P.group_gpos[k] = (uint32_t)li[gq[k]];
            P.group_gpos[m + k] = (uint32_t)li[gq[k] + n];
            P.out_gpos[k] = (uint32_t)lo[gq[k]];
            P.out_gpos[m + k] = (uint32_t)lo[gq[k] + n];
        }
        // launch blocks over the group qubits with a bit below position 3
        // in the loaded layout (they split 128-byte lines between tiles)
        uint32_t c = 0;
        while (c < m && std::min(li[gq[c]], li[gq[c] + n]) < 3) ++c;
        const uint64_t N = 1ull << m, NB = N >> c, NBB = NB * (NB + 1) / 2;
        const uint32_t stride = (uint32_t)std::min<uint64_t>(8, NBB);
        P.n_tiles = (NBB + stride - 1) / stride * stride << (2 * c);
        P.herm = (P.herm & (kHermHalfIn | kHermMirror)) | kHermPass | (c << kHermLineShift) |
                 (stride << kHermStrideShift);
        const uint32_t nthr = P.L - 4;
        for (uint32_t ph = P.phase_begin; ph < P.phase_end; ++ph) {
            KPhase &H = plan.phases[ph];
            const bool last = ph + 1 == P.phase_end && P.phase_end - P.phase_begin > 1;
            const Layout &lh = last ? lo : li;
            place_phase(H, nthr, lh, n);
            for (uint32_t oi = H.op_begin; oi < H.op_end; ++oi) {
                KOp &o = plan.ops[oi];
                if (o.kind == KOP_DIAG_RT)
                    for (uint32_t j = 0; j < o.nbits; ++j) o.gpos[j] = (uint32_t)li[o.gpos[j]];
            }
        }
        coalesce_lanes(plan.phases[P.phase_begin], nthr, li, n);
        if (P.phase_end - P.phase_begin > 1) coalesce_lanes(plan.phases[P.phase_end - 1], nthr, lo, n);
    }
    plan.relabelled = true;
    return io_ok;
}

// Qubits of a Hermitian pass's tile (logical positions: before relabelling).
uint32_t pass_tile(const KPass &P, int n)
{
    const uint32_t m = P.n_group_bits >> 1;
    uint32_t g = 0;
    for (uint32_t k = 0; k < m; ++k) g |= 1u << P.group_gpos[k];
    return ((1u << n) - 1u) & ~g;
}

// Qubits with a bit among a phase's register bits.
uint32_t reg_qubits(const KPhase &H, int n)
{
    uint32_t m = 0;
    for (int b = 0; b < kRegBits; ++b)
        if (H.reg_gpos[b] < 2u * (uint32_t)n) m |= 1u << (H.reg_gpos[b] % (uint32_t)n);
    return m;
}

// Tile-local bit positions are labels of the LDS layout alone, so a pass
// may permute them (every phase's register and thread positions and the
// local positions of its runtime-diagonal ops together).  The permutation
// puts lanes 0-3 of the phase that loads HBM on tile bits of residues
// 0, 1, 2, 3 (mod 4), and the lanes of the phase that stores HBM on
// distinct residues too, where possible: their lane order is fixed by the
// global accesses, and under the LDS swizzle tile bit p lands in bank-group
// bit p mod 4.
void relabel_tile_bits(HostPlan &plan)
{
    for (const KPass &P : plan.passes) {
        if (P.phase_end - P.phase_begin < 2) continue;
        const uint32_t L = P.L, nthr = L - 4, nl = nthr < 4 ? nthr : 4;
        const KPhase &F = plan.phases[P.phase_begin], &S = plan.phases[P.phase_end - 1];
        std::vector<int> colour(L, -1);
        for (uint32_t j = 0; j < nl; ++j) colour[F.thr_local[j]] = (int)j;
        std::vector<bool> used_b(4, false);
        for (uint32_t j = 0; j < nl; ++j)
            if (colour[S.thr_local[j]] >= 0) used_b[colour[S.thr_local[j]]] = true;
        for (uint32_t j = 0; j < nl; ++j) {
            const uint32_t p = S.thr_local[j];
            if (colour[p] >= 0) continue;
            for (int c = 0; c < 4; ++c)
                if (!used_b[c]) {
                    colour[p] = c;
                    used_b[c] = true;
                    break;
                }
        }
        // pi: coloured positions first (lane order of the load phase, then
        // of the store phase), each to the lowest free target of its residue
        std::vector<int> pi(L, -1);
        std::vector<bool> taken(L, false);
        auto place = [&](uint32_t p) {
            if (pi[p] >= 0 || colour[p] < 0) return;
            for (uint32_t t = (uint32_t)colour[p]; t < L; t += 4)
                if (!taken[t]) {
                    pi[p] = (int)t;
                    taken[t] = true;
                    return;
                }
        };
        for (uint32_t j = 0; j < nl; ++j) place(F.thr_local[j]);
        for (uint32_t j = 0; j < nl; ++j) place(S.thr_local[j]);
        uint32_t next = 0;
        for (uint32_t p = 0; p < L; ++p) {
            if (pi[p] >= 0) continue;
            while (taken[next]) ++next;
            pi[p] = (int)next;
            taken[next] = true;
        }
        for (uint32_t ph = P.phase_begin; ph < P.phase_end; ++ph) {
            KPhase &H = plan.phases[ph];
            for (int b = 0; b < kRegBits; ++b) H.reg_local[b] = (uint32_t)pi[H.reg_local[b]];
            for (uint32_t t = 0; t < nthr; ++t) H.thr_local[t] = (uint32_t)pi[H.thr_local[t]];
            for (uint32_t oi = H.op_begin; oi < H.op_end; ++oi) {
                KOp &o = plan.ops[oi];
                if (o.kind != KOP_DIAG_RT) continue;
                for (uint32_t j = 0; j < o.nbits; ++j)
                    if (o.lpos[j] != kNotLocal) o.lpos[j] = (uint32_t)pi[o.lpos[j]];
            }
        }
    }
}

// Lane order of the phases that neither load nor store HBM (their thread
// bits may be permuted freely: an exchange addresses LDS by tile-local index
// alone).  The LDS index swizzle xors the three nibbles of the tile-local
// index into the low one, so tile bit p lands in bank-group bit p mod 4
// (16-byte groups).  Lanes 0-2 take thread bits of residues 0, 1, 2 and lane
// 3 one of residue 3, where the phase has them: then the 16 lanes of a
// 128-bit LDS access (or any 8 of them) hit distinct bank groups.
void spread_lane_banks(HostPlan &plan)
{
    for (const KPass &P : plan.passes) {
        const uint32_t nthr = P.L - 4;
        for (uint32_t ph = P.phase_begin + 1; ph + 1 < P.phase_end; ++ph) {
            KPhase &H = plan.phases[ph];
            std::vector<uint32_t> order;
            std::vector<bool> used(nthr, false);
            for (uint32_t r = 0; r < 4 && r < nthr; ++r)
                for (uint32_t t = 0; t < nthr; ++t)
                    if (!used[t] && H.thr_local[t] % 4 == r) {
                        order.push_back(t);
                        used[t] = true;
                        break;
                    }
            for (uint32_t t = 0; t < nthr; ++t)
                if (!used[t]) order.push_back(t);
            const KPhase old = H;
            for (uint32_t t = 0; t < nthr; ++t) {
                H.thr_local[t] = old.thr_local[order[t]];
                H.thr_gpos[t] = old.thr_gpos[order[t]];
                H.thr_mpos[t] = old.thr_mpos[order[t]];
            }
        }
    }
}

}  // namespace

// share_mode (Hermitian plans with relabelled layouts): instead of keeping
// qubits 0..hc-1 in every tile, each tile keeps a qubit of the previous
// tile that the previous pass's storing phase holds outside its registers,
// and the loading phase is padded only where that qubit would be in its
// registers; the relabelled layout between the two passes leads with it.
// Returns kPlanRetry when some pass's I/O would still start in a register.
constexpr int kPlanRetry = 1;

int plan_program_mode(int n, const std::vector<LOp> &ops, const PlanOpts &opt, HostPlan &out, bool share_mode)
{
    out = HostPlan{};
    const int n2 = 2 * n;
    if (opt.tile_bits < 4 || opt.tile_bits > kMaxTileBits)
        return fail(VQD_E_ARG, "tile_bits must be in [4, 13]");
    // tile size actually used: 2n bits at most, but never fewer than the 4
    // register bits (tiny registers get phantom bits)
    // Hermitian mode: tiles are whole qubits (row and column bit), so the
    // tile size is even; qubits 0..hc-1 are in every tile so that the loads,
    // the stores and the mirrored stores all cover 2^hc contiguous amplitudes
    bool herm = opt.hermitian && n >= 2;
    for (size_t i = 0; herm && i < ops.size(); ++i) herm = preserves_hermiticity(ops[i]);
    out.hermitian = herm;
    const int L = herm ? std::min(opt.tile_bits & ~1, n2) : std::max(4, std::min(opt.tile_bits, n2));
    const int contig = std::max(0, std::min(opt.min_contig_bits, std::min(L, n2)));
    // (fewer when the program's widest non-diagonal op would not fit beside them)
    int kmax = 1;
    for (const LOp &op : ops)
        if (!op.diag) kmax = std::max(kmax, op.k);
    const int hc = (herm && !share_mode) ? std::max(0, std::min(std::min(std::min(contig, 3), n), L / 2 - kmax)) : 0;
    const uint32_t forced = (1u << hc) - 1u;        // qubits in every Hermitian tile
    const int max_take = opt.max_ops_per_pass;
    // LDS left for the runtime-diagonal tables beside the staged tile
    const size_t rt_budget = opt.rt_budget > 0 ? (size_t)opt.rt_budget
                                               : (size_t(160 * 1024) - 1024 - (size_t(16) << L)) / 16;

    std::vector<uint32_t> qm(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) {
        qm[i] = qmask(ops[i]);
        const int need = (int)tile_bits_for(qm[i], n, 0).size();
        if (!ops[i].diag && need > L)
            return fail(VQD_E_SIZE, "op " + std::to_string(i) + " needs " + std::to_string(need) +
                                        " tile bits; tile has " + std::to_string(L));
    }

    // exact identities (e.g. a zero-probability channel) are dropped
    std::vector<char> applied(ops.size(), 0);
    for (size_t i = 0; i < ops.size(); ++i) {
        const LOp &op = ops[i];
        if (!op.diag || op.wide_unitary) continue;
        bool ident = true;
        for (const cd &f : op.D)
            if (f != cd(1)) { ident = false; break; }
        if (ident && !opt.keep_identity) applied[i] = 1;
    }
    size_t first = 0;
    SimResult sim, sim2;
    int retry_take = 0;     // > 0: the last attempt at this pass overflowed LDS
    // share_mode: the previous tile's qubits outside its storing registers
    // (before the first pass: qubit 0, which leads the caller's layout)
    uint32_t prev_free = share_mode ? 1u : 0u;
    while (true) {
        while (first < ops.size() && applied[first]) ++first;
        if (first >= ops.size()) break;
        const int take_cap = retry_take > 0 ? retry_take : max_take;

        // ---- choose the pass qubit set
        uint32_t Q = herm ? forced : 0u;
        while (true) {
            simulate(ops, qm, applied, first, Q, n, take_cap, sim, true);
            const size_t base = sim.taken.size();
            if (take_cap > 0 && (int)base >= take_cap) break;
            uint32_t bestQ = Q;
            size_t bestc = base;
            for (uint32_t c : sim.cands) {
                const uint32_t Q2 = Q | c;
                // the contiguous low bits are a preference: the first op of a
                // pass may use them when it cannot fit otherwise
                const int reserve = (share_mode && prev_free && !(Q2 & prev_free)) ? 2 : 0;
                const bool fits = herm ? (int)tile_bits_for(Q2 | forced, n, 0).size() + reserve <= L
                                       : ((int)tile_bits_for(Q2, n, contig).size() <= L ||
                                          (Q == 0 && (int)tile_bits_for(Q2, n, 0).size() <= L));
                if (!fits) continue;
                simulate(ops, qm, applied, first, Q2, n, take_cap, sim2, false);
                if (sim2.taken.size() > bestc) {
                    bestc = sim2.taken.size();
                    bestQ = Q2;
                }
            }
            if (bestQ == Q) break;
            Q = bestQ;
        }
        if (share_mode && prev_free && !(Q & prev_free) && popc(Q) < L / 2)
            Q |= 1u << __builtin_ctz(prev_free);
        if (herm)      // the tile's filler qubits are the lowest others: ops on them may join too
            for (int q = 0; popc(Q) < L / 2 && q < n; ++q) Q |= 1u << q;
        simulate(ops, qm, applied, first, Q, n, take_cap, sim, false);
        if (sim.taken.empty()) return fail(VQD_E_STATE, "planner made no progress");
        for (int i : sim.taken) applied[i] = 1;
        const size_t ops_before = out.ops.size(), mats_before = out.mats.size(),
                     recipes_before = out.recipes.size();

        // ---- tile bits
        std::vector<int> tb;
        uint32_t tq = 0;                              // Hermitian mode: the tile's qubits
        if (herm) {
            tq = Q | forced;
            for (int q = 0; popc(tq) < L / 2 && q < n; ++q) tq |= 1u << q;
            tb = tile_bits_for(tq, n, 0);
        } else {
            tb = tile_bits_for(Q, n, contig);
            if ((int)tb.size() > L) tb = tile_bits_for(Q, n, 0);
            for (int b = 0; (int)tb.size() < std::min(L, n2) && b < n2; ++b)
                if (std::find(tb.begin(), tb.end(), b) == tb.end()) tb.push_back(b);
            std::sort(tb.begin(), tb.end());
            for (uint32_t ph = kPhantomPos; (int)tb.size() < L; ++ph) tb.push_back((int)ph);  // phantom bits (tiny n)
        }
        KPass kp{};
        kp.L = (uint32_t)L;
        kp.phantom = (n2 < L) ? 1u : 0u;
        int ng = 0;
        if (herm) {
            // the m group qubits' row bits, then their column bits in the same order
            std::vector<int> gq;
            for (int q = 0; q < n; ++q)
                if (!(tq >> q & 1)) gq.push_back(q);
            for (int q : gq) kp.group_gpos[ng++] = (uint32_t)q;
            for (int q : gq) kp.group_gpos[ng++] = (uint32_t)(q + n);
            // group qubits below 3 split 128-byte lines: the lowest group
            // bits, launched in blocks (ascending order puts them first)
            uint32_t c = 0;
            while (c < gq.size() && gq[c] < 3) ++c;
            const uint64_t N = 1ull << gq.size(), NB = N >> c, NBB = NB * (NB + 1) / 2;
            const uint32_t stride = (uint32_t)std::min<uint64_t>(8, NBB);
            kp.n_tiles = (NBB + stride - 1) / stride * stride << (2 * c);
            kp.herm = kHermPass | (c << kHermLineShift) | (stride << kHermStrideShift);
            out.tile_fraction = double(N + 1) / double(2 * N);
        } else {
            for (int b = 0; b < n2; ++b)
                if (std::find(tb.begin(), tb.end(), b) == tb.end()) kp.group_gpos[ng++] = (uint32_t)b;
            kp.n_tiles = 1ull << ng;
        }
        kp.n_group_bits = (uint32_t)ng;
        // tiles lacking the lowest vector bits share cache lines with their
        // neighbours in the low group bits; keep those on one XCD
        bool low_in_tile = true;
        for (int b = 0; b < std::min(3, n2); ++b)
            if (std::find(tb.begin(), tb.end(), b) == tb.end()) low_in_tile = false;
        kp.xcd_swizzle = (!herm && !low_in_tile && kp.n_tiles >= 64 && kp.n_tiles % 64 == 0) ? 1u : 0u;
        kp.phase_begin = (uint32_t)out.phases.size();
        const double fma_before = out.fma_per_amp;
        std::vector<cd> rt_tables;      // runtime-diagonal tables of this pass (LDS-staged)
        auto local_of = [&](int g) {
            for (int i = 0; i < (int)tb.size(); ++i)
                if (tb[i] == g) return i;
            return -1;
        };

        // ---- phases
        auto emit_phase = [&](const int *reg_gpos, const std::vector<Block> &blocks,
                              const std::vector<int> &rt_ops_unused) {
            (void)rt_ops_unused;
            KPhase H{};
            bool used[kMaxTileBits] = {false};
            for (int b = 0; b < 4; ++b) {
                const int l = local_of(reg_gpos[b]);
                H.reg_local[b] = (uint32_t)l;
                H.reg_gpos[b] = (uint32_t)reg_gpos[b];
                used[l] = true;
            }
            // thread bits: the first three (lanes 0..7 of a wave) take one free
            // local bit from each residue class mod 3, so that the LDS swizzle
            // (low three bits xor bits 3-5, 6-8, 9-11) spreads every group of 8
            // lanes over all banks; the rest follow in ascending order
            std::vector<int> tl_order;
            for (int cls = 0; cls < 3; ++cls)
                for (int l = 0; l < L; ++l)
                    if (!used[l] && l % 3 == cls) {
                        tl_order.push_back(l);
                        break;
                    }
            if ((int)tl_order.size() < 3) tl_order.clear();
            std::sort(tl_order.begin(), tl_order.end());
            for (int l = 0; l < L; ++l)
                if (!used[l] && std::find(tl_order.begin(), tl_order.end(), l) == tl_order.end())
                    tl_order.push_back(l);
            for (int t = 0; t < L - 4; ++t) {
                H.thr_local[t] = (uint32_t)tl_order[t];
                H.thr_gpos[t] = (uint32_t)tb[tl_order[t]];
            }
            H.op_begin = (uint32_t)out.ops.size();
            // Runtime diagonals: a run of consecutive ones (all diagonal, so
            // they commute) is regrouped by register pair and each group is
            // tabulated as one op over the union of its gathered bits.
            auto rt_part = [&](int op_index) {
                const LOp &op = ops[op_index];
                const int nb = 2 * op.k;
                RtPart pt;
                pt.src = op_index;
                int sb[4];
                for (int j = 0; j < nb; ++j) {
                    pt.g[j] = (j < op.k) ? op.q[j] : op.q[j - op.k] + n;
                    sb[j] = -1;
                    for (int b = 0; b < 4; ++b)
                        if (reg_gpos[b] == pt.g[j]) sb[j] = b;
                }
                pt.nb = nb;
                std::vector<int> regj;
                for (int j = 0; j < nb; ++j) (sb[j] >= 0 ? regj : pt.rtj).push_back(j);
                pt.mode = RT_GENERIC;
                if (regj.empty()) {
                    pt.mode = RT_NONE;
                } else if (regj.size() == 2) {
                    for (int j : regj) {
                        if (sb[j] == 0 || sb[j] == 1) pt.row_j = j;
                        if (sb[j] == 2 || sb[j] == 3) pt.col_j = j;
                    }
                    if (pt.row_j >= 0 && pt.col_j >= 0 && sb[pt.col_j] == sb[pt.row_j] + 2)
                        pt.mode = sb[pt.row_j] == 0 ? RT_PAIR_A : RT_PAIR_B;
                }
                if (pt.mode == RT_GENERIC) {
                    pt.rtj.clear();
                    for (int j = 0; j < nb; ++j) pt.rtj.push_back(j);
                    pt.row_j = pt.col_j = -1;
                }
                return pt;
            };
            auto emit_rt = [&](uint32_t mode, std::vector<RtPart> parts) {
                KOp ko{};
                ko.kind = KOP_DIAG_RT;
                ko.mode = mode;
                std::vector<int> ubits;                  // union of gathered global bits
                for (RtPart &pt : parts) {
                    pt.upos.clear();
                    for (int j : pt.rtj) {
                        const int gg = pt.g[j];
                        auto it = std::find(ubits.begin(), ubits.end(), gg);
                        if (it == ubits.end()) {
                            pt.upos.push_back((int)ubits.size());
                            ubits.push_back(gg);
                        } else {
                            pt.upos.push_back((int)(it - ubits.begin()));
                        }
                    }
                }
                ko.nbits = (uint32_t)ubits.size();
                for (size_t j = 0; j < ubits.size(); ++j) {
                    ko.gpos[j] = (uint32_t)ubits[j];
                    const int l = local_of(ubits[j]);
                    ko.lpos[j] = (l >= 0) ? (uint32_t)l : kNotLocal;
                }
                std::vector<cd> table;
                rt_table(mode, (int)ubits.size(), parts, ops, table);
                ko.real = all_real(table) ? 1u : 0u;
                ko.mat = (uint32_t)rt_tables.size();
                rt_tables.insert(rt_tables.end(), table.begin(), table.end());
                out.fma_per_amp += ko.real ? 2.0 : 4.0;
                if (opt.record_recipes) {
                    Recipe r;
                    r.rt = true;
                    for (const RtPart &pt : parts) r.src.push_back(pt.src);
                    r.kind = KOP_DIAG_RT;
                    r.real = ko.real != 0;
                    r.mode = mode;
                    r.rt_union = (int)ubits.size();
                    r.rt_parts = parts;
                    r.mat_off = ko.mat;      // made absolute when the pass closes
                    out.recipes.push_back(r);
                }
                out.ops.push_back(ko);
            };
            for (size_t bi = 0; bi < blocks.size();) {
                const Block &bk = blocks[bi];
                if (bk.rt) {
                    size_t be = bi;
                    while (be < blocks.size() && blocks[be].rt) ++be;
                    std::vector<RtPart> groups[3];     // pair A, pair B, none
                    for (size_t k = bi; k < be; ++k) {
                        RtPart pt = rt_part(blocks[k].op_index);
                        if (pt.mode == RT_GENERIC) emit_rt(RT_GENERIC, {pt});
                        else groups[pt.mode == RT_PAIR_A ? 0 : pt.mode == RT_PAIR_B ? 1 : 2].push_back(pt);
                    }
                    // index-only factors join a pair group when there is one
                    const int host = !groups[0].empty() ? 0 : !groups[1].empty() ? 1 : 2;
                    if (host != 2) {
                        groups[host].insert(groups[host].end(), groups[2].begin(), groups[2].end());
                        groups[2].clear();
                    }
                    const uint32_t gmode[3] = {RT_PAIR_A, RT_PAIR_B, RT_NONE};
                    for (int gi = 0; gi < 3; ++gi) {
                        std::vector<RtPart> chunk;
                        std::vector<int> cu;
                        for (const RtPart &pt : groups[gi]) {
                            std::vector<int> u2 = cu;
                            for (int j : pt.rtj)
                                if (std::find(u2.begin(), u2.end(), pt.g[j]) == u2.end()) u2.push_back(pt.g[j]);
                            if (!chunk.empty() && ((int)u2.size() > kMaxRtBits || !opt.merge_rt)) {
                                emit_rt(gmode[gi], chunk);
                                chunk.clear();
                                cu.clear();
                                for (int j : pt.rtj) cu.push_back(pt.g[j]);
                            } else {
                                cu = u2;
                            }
                            chunk.push_back(pt);
                        }
                        if (!chunk.empty()) emit_rt(gmode[gi], chunk);
                    }
                    bi = be;
                    continue;
                }
                KOp ko{};
                {
                    Encoded enc = encode(bk.m);
                    if (enc.identity) {
                        if (!opt.keep_identity) {
                            ++bi;
                            continue;
                        }
                        // a template keeps the slot: other parameters need not give 1
                        enc.kind = KOP_DIAG;
                        enc.mask = 15;
                        enc.real = true;
                        enc.data = pack(std::vector<cd>(16, cd(1)), true);
                        enc.cost = 32.0;
                    }
                    ko.kind = enc.kind;
                    ko.opmask = (uint32_t)enc.mask;
                    ko.real = enc.real ? 1u : 0u;
                    ko.mat = (uint32_t)out.mats.size();
                    out.mats.insert(out.mats.end(), enc.data.begin(), enc.data.end());
                    out.fma_per_amp += enc.cost / 16.0;
                    if (opt.record_recipes) {
                        Recipe r;
                        r.src = bk.src;
                        for (int b = 0; b < 4; ++b) r.reg_gpos[b] = reg_gpos[b];
                        r.kind = enc.kind;
                        r.mask = (uint32_t)enc.mask;
                        r.real = enc.real;
                        r.mat_off = ko.mat;
                        if (bk.wide_half >= 0) r.mode = 100u + (uint32_t)bk.wide_half;
                        out.recipes.push_back(r);
                    }
                }
                out.ops.push_back(ko);
                ++bi;
            }
            H.op_end = (uint32_t)out.ops.size();
            out.phases.push_back(H);
        };

        // filler register bits: highest tile bits not otherwise used
        // filler register bits: the highest tile bits not otherwise used,
        // preferring bits that no runtime-diagonal op of the phase reads
        auto fill_regs = [&](int *reg, const std::vector<int> &fixed_idx,
                             const std::vector<int> &prefer_not) {
            std::vector<int> taken;
            for (int b : fixed_idx) taken.push_back(reg[b]);
            std::vector<int> order;          // candidate tile bits, best first
            for (int li = L - 1; li >= 0; --li)
                if (std::find(prefer_not.begin(), prefer_not.end(), tb[li]) == prefer_not.end())
                    order.push_back(tb[li]);
            for (int li = L - 1; li >= 0; --li)
                if (std::find(prefer_not.begin(), prefer_not.end(), tb[li]) != prefer_not.end())
                    order.push_back(tb[li]);
            size_t oi = 0;
            for (int b = 0; b < 4; ++b) {
                if (std::find(fixed_idx.begin(), fixed_idx.end(), b) != fixed_idx.end()) continue;
                while (std::find(taken.begin(), taken.end(), order[oi]) != taken.end()) ++oi;
                reg[b] = order[oi];
                taken.push_back(order[oi]);
            }
        };

        std::vector<int> rem = sim.taken;
        while (!rem.empty()) {
            uint32_t P = 0;
            std::vector<int> take, keep;
            uint32_t blk_any = 0, blk_nd = 0;
            int wide = -1;
            for (int idx : rem) {
                const LOp &op = ops[idx];
                const uint32_t m = qm[idx];
                bool ok = false;
                if (wide >= 0) {
                    ok = false;
                } else if (m & blk_any) {
                } else if (!op.diag && (m & blk_nd)) {
                } else if (op.diag) {
                    ok = true;
                } else if (op.wide_unitary) {
                    if (P == 0) {
                        bool nd_taken = false;
                        for (int t : take) nd_taken |= !ops[t].diag;
                        if (!nd_taken) { ok = true; wide = idx; P = m; }
                    }
                } else if ((m & ~P) == 0) {
                    ok = true;
                } else if (popc(P | m) <= 2) {
                    P |= m;
                    ok = true;
                }
                if (ok) {
                    take.push_back(idx);
                } else {
                    keep.push_back(idx);
                    if (op.diag) blk_nd |= m;
                    else blk_any |= m;
                }
            }
            rem.swap(keep);

            if (wide >= 0) {
                // diagonal ops taken before the wide op go into the row phase
                const LOp &w = ops[wide];
                const int k = w.k, d = 1 << k;
                for (int half = 0; half < 2; ++half) {
                    int reg[4];
                    std::vector<int> fixed;
                    for (int j = 0; j < k; ++j) {
                        reg[j] = w.q[j] + (half ? n : 0);
                        fixed.push_back(j);
                    }
                    fill_regs(reg, fixed, {});
                    std::vector<Block> blocks;
                    if (half == 0)
                        for (int idx : take)
                            if (idx != wide) {
                                Block bk;
                                bk.rt = true;
                                bk.op_index = idx;
                                blocks.push_back(bk);
                            }
                    // matrix on register bits 0..k-1 (mask 7 or 15), embedded
                    Mat16 m{};
                    const int mask = (1 << k) - 1, rest = (~mask) & 15;
                    for (int so = 0; so < 16; ++so)
                        for (int si = 0; si < 16; ++si) {
                            if ((so & rest) != (si & rest)) continue;
                            const cd u = w.U[size_t(so & mask) * d + (si & mask)];
                            m[so * 16 + si] = half ? std::conj(u) : u;
                        }
                    Block bk;
                    bk.m = m;
                    bk.src = {wide};
                    bk.wide_half = half;
                    blocks.push_back(bk);
                    emit_phase(reg, blocks, {});
                }
                continue;
            }

            // register bits: [qa, qb, qa+n, qb+n] (fillers when fewer qubits)
            int reg[4];
            std::vector<int> fixed;
            int qs[2], nq = 0;
            for (int q = 0; q < n && nq < 2; ++q)
                if (P >> q & 1) qs[nq++] = q;
            if (nq >= 1) { reg[0] = qs[0]; reg[2] = qs[0] + n; fixed.push_back(0); fixed.push_back(2); }
            if (nq == 2) { reg[1] = qs[1]; reg[3] = qs[1] + n; fixed.push_back(1); fixed.push_back(3); }
            std::vector<int> rt_bits;           // bits read by this phase's runtime diagonals
            for (int idx : take) {
                const LOp &op = ops[idx];
                if (op.diag && (qm[idx] & ~P) != 0)
                    for (int j = 0; j < op.k; ++j) {
                        rt_bits.push_back(op.q[j]);
                        rt_bits.push_back(op.q[j] + n);
                    }
            }
            fill_regs(reg, fixed, rt_bits);

            // blocks in order, fusing across commuting blocks where cheaper
            std::vector<Block> blocks;
            for (int idx : take) {
                const LOp &op = ops[idx];
                const uint32_t m = qm[idx];
                if (op.diag && (m & ~P) != 0) {
                    Block bk;
                    bk.rt = true;
                    bk.op_index = idx;
                    blocks.push_back(bk);
                    continue;
                }
                Block nb;
                nb.m = embed(op, n, reg, nb.support);
                nb.diag = op.diag;
                nb.src = {idx};
                bool merged = false;
                if (opt.fuse_blocks) {
                    for (int j = (int)blocks.size() - 1; j >= 0; --j) {
                        Block &pb = blocks[j];
                        if (pb.rt) break;
                        // blocks on disjoint register bits commute: look further back
                        if ((pb.support & nb.support) == 0) continue;
                        // first overlapping block: fuse with it if that is cheaper
                        Mat16 prod = mul(nb.m, pb.m);
                        const double cp = encode(prod).cost;
                        if (cp <= encode(pb.m).cost + encode(nb.m).cost) {
                            pb.m = prod;
                            pb.support |= nb.support;
                            pb.diag = pb.diag && nb.diag;
                            pb.src.insert(pb.src.end(), nb.src.begin(), nb.src.end());
                            merged = true;
                        }
                        break;
                    }
                }
                if (!merged) blocks.push_back(nb);
            }
            emit_phase(reg, blocks, {});
        }
        // The first phase's register mapping also serves the HBM loads and the
        // last one's the stores.  If a register bit is one of the lowest
        // (contiguous) vector bits, lanes would stride; an op-free phase on
        // high tile bits is added instead (an LDS exchange is cheaper).
        if (herm && L - 4 >= 2 * hc) {
            // Hermitian mode: the loads (first phase), the stores and the
            // mirrored stores (last phase) are coalesced when the local bits of
            // global bits 0..hc-1 and n..n+hc-1 are the lowest thread bits, in
            // that order; an op-free phase is added where a register holds one
            std::vector<int> io_local, io_gpos;
            for (int q = 0; q < hc; ++q) io_gpos.push_back(q);
            for (int q = 0; q < hc; ++q) io_gpos.push_back(q + n);
            for (int g : io_gpos) io_local.push_back(local_of(g));
            auto io_in_regs = [&](const KPhase &H) {
                for (int b = 0; b < 4; ++b)
                    if (std::find(io_local.begin(), io_local.end(), (int)H.reg_local[b]) != io_local.end())
                        return true;
                return false;
            };
            const size_t first_ph = kp.phase_begin;
            bool pad_front = io_in_regs(out.phases[first_ph]);
            bool pad_back = io_in_regs(out.phases.back());
            std::vector<int> avoid = io_gpos, avoid_back = io_gpos;
            if (share_mode) {
                // the loading phase must leave a shared free qubit out of its
                // registers (qubit 0 for the first pass, which loads the
                // caller's layout); the last pass stores the caller's layout,
                // led by qubit 0
                const uint32_t S = tq & prev_free;
                pad_front = S && !(S & ~reg_qubits(out.phases[first_ph], n));
                if (pad_front) avoid = {__builtin_ctz(S), __builtin_ctz(S) + n};
                bool last_pass = true;
                for (size_t i = first; i < ops.size() && last_pass; ++i) last_pass = applied[i] != 0;
                pad_back = last_pass && (reg_qubits(out.phases.back(), n) & 1u);
                avoid_back = {0, n};
                // a pass with one phase would load and store through the same
                // registers and keep its layout: give it a storing phase of
                // its own, so that every boundary gets its relabelled layout
                if (out.phases.size() - first_ph == 1) pad_back = true;
            }
            if (pad_front || pad_back) {
                const std::vector<Block> none;
                if (pad_back) {
                    int reg[4];
                    fill_regs(reg, {}, avoid_back);
                    emit_phase(reg, none, {});
                }
                if (pad_front) {
                    int reg[4];
                    fill_regs(reg, {}, avoid);
                    const uint32_t ob = out.phases[first_ph].op_begin;
                    emit_phase(reg, none, {});
                    KPhase dummy = out.phases.back();
                    dummy.op_begin = dummy.op_end = ob;
                    out.phases.pop_back();
                    out.phases.insert(out.phases.begin() + first_ph, dummy);
                }
            }
            auto io_first = [&](KPhase &H) {
                std::vector<uint32_t> order(io_local.begin(), io_local.end());
                for (int t = 0; t < L - 4; ++t)
                    if (std::find(io_local.begin(), io_local.end(), (int)H.thr_local[t]) == io_local.end())
                        order.push_back(H.thr_local[t]);
                for (int t = 0; t < L - 4; ++t) {
                    H.thr_local[t] = order[t];
                    H.thr_gpos[t] = (uint32_t)tb[order[t]];
                }
            };
            io_first(out.phases[first_ph]);
            io_first(out.phases.back());
        } else if (!herm) {
            const int low = std::min(3, std::min(contig, n2));
            auto strided = [&](const KPhase &H) {
                for (int b = 0; b < 4; ++b)
                    if ((int)H.reg_gpos[b] < low) return true;
                return false;
            };
            const size_t first_ph = kp.phase_begin;
            // only for light passes: in a pass dominated by FP64 work the
            // strided access is hidden and the extra exchange is not
            const bool light = (out.fma_per_amp - fma_before) < 32.0;
            const bool pad_front = opt.pad_coalesce && light && low > 0 && out.phases.size() > first_ph && strided(out.phases[first_ph]);
            const bool pad_back = opt.pad_coalesce && light && low > 0 && out.phases.size() > first_ph && strided(out.phases.back());
            if (pad_front || pad_back) {
                int reg[4];
                fill_regs(reg, {}, {});
                const std::vector<Block> none;
                if (pad_back) emit_phase(reg, none, {});
                if (pad_front) {
                    const uint32_t ob = out.phases[first_ph].op_begin;
                    emit_phase(reg, none, {});
                    KPhase dummy = out.phases.back();
                    dummy.op_begin = dummy.op_end = ob;
                    out.phases.pop_back();
                    out.phases.insert(out.phases.begin() + first_ph, dummy);
                }
            }
        }
        if (rt_tables.size() > rt_budget) {
            // too many tables to stage: undo the pass and take half the ops
            if (sim.taken.size() <= 1) return fail(VQD_E_SIZE, "a diagonal op's table exceeds the LDS budget");
            out.phases.resize(kp.phase_begin);
            out.ops.resize(ops_before);
            out.mats.resize(mats_before);
            out.recipes.resize(recipes_before);
            out.fma_per_amp = fma_before;
            for (int i : sim.taken) applied[i] = 0;
            retry_take = (int)sim.taken.size() / 2;
            continue;
        }
        retry_take = 0;
        kp.phase_end = (uint32_t)out.phases.size();
        kp.rt_mat = (uint32_t)out.mats.size();
        kp.rt_count = (uint32_t)rt_tables.size();
        if (opt.record_recipes)
            for (uint32_t oi = out.phases[kp.phase_begin].op_begin; oi < out.ops.size(); ++oi)
                if (out.recipes[oi].rt) out.recipes[oi].mat_off += kp.rt_mat;
        out.mats.insert(out.mats.end(), rt_tables.begin(), rt_tables.end());
        std::copy(kp.group_gpos, kp.group_gpos + 32, kp.out_gpos);   // the layout stays
        kp.swap_out = 0;
        out.passes.push_back(kp);
        if (share_mode) prev_free = pass_tile(kp, n) & ~reg_qubits(out.phases[kp.phase_end - 1], n);
    }
    if (herm) {
        // between the passes of a program only the computed half is stored;
        // the last pass restores the whole matrix
        for (size_t i = 0; i < out.passes.size(); ++i) {
            if (i > 0) out.passes[i].herm |= kHermHalfIn;
            if (i + 1 == out.passes.size()) out.passes[i].herm |= kHermMirror;
        }
        if (opt.relayout && !relabel_passes(n, out) && share_mode) return kPlanRetry;
    }
    relabel_tile_bits(out);
    spread_lane_banks(out);
    finish_slot_tables(n, out);
    return VQD_OK;
}

int plan_program(int n, const std::vector<LOp> &ops, const PlanOpts &opt, HostPlan &out)
{
    if (opt.relayout && opt.hermitian) {
        const int rc = plan_program_mode(n, ops, opt, out, true);
        if (rc != kPlanRetry) return rc;
    }
    return plan_program_mode(n, ops, opt, out, false);
}

void finish_slot_tables(int n, HostPlan &plan)
{
    for (KPhase &H : plan.phases) {
        if (!plan.relabelled) {
            // the vectorised layout throughout
            for (int b = 0; b < kRegBits; ++b) H.reg_mpos[b] = mirror_pos(H.reg_gpos[b], (uint32_t)n) & 31u;
            for (int t = 0; t < kMaxThreadBits; ++t) H.thr_mpos[t] = mirror_pos(H.thr_gpos[t], (uint32_t)n) & 31u;
        }
        for (int e = 0; e < kSlots; ++e) {
            uint32_t l = 0, g = 0, gm = 0;
            for (int b = 0; b < kRegBits; ++b)
                if (e >> b & 1) {
                    l |= 1u << (H.reg_local[b] & 31u);
                    g |= 1u << (H.reg_gpos[b] & 31u);
                    gm |= 1u << (H.reg_mpos[b] & 31u);
                }
            H.lds_slot[e] = lds_swizzle(l) << 4;
            H.g_slot[e] = g;
            H.gm_slot[e] = gm;
        }
    }
    for (size_t p = 0; p < plan.passes.size(); ++p) {
        KPass &P = plan.passes[p];
        std::fill(P.hi_slot, P.hi_slot + kSlots, 0u);
        std::fill(P.hj_slot, P.hj_slot + kSlots, 0u);
        if (!(P.herm & kHermHalfIn) || p == 0) continue;
        // the bits of slot e's index, taken at the previous pass's row
        // (i) and column (j) group positions in the layout it stored
        const KPass &Q = plan.passes[p - 1];
        const KPhase &H0 = plan.phases[P.phase_begin];
        const uint32_t m = Q.n_group_bits >> 1;
        for (int e = 0; e < kSlots; ++e) {
            const uint32_t x = H0.g_slot[e];
            uint32_t i = 0, j = 0;
            for (uint32_t k = 0; k < m; ++k) {
                i |= ((x >> (Q.out_gpos[k] & 31u)) & 1u) << k;
                j |= ((x >> (Q.out_gpos[m + k] & 31u)) & 1u) << k;
            }
            P.hi_slot[e] = i;
            P.hj_slot[e] = j;
        }
    }
}

namespace {

bool same_targets(const LOp &x, const LOp &y)
{
    if (x.k != y.k || x.wide_unitary || y.wide_unitary) return false;
    for (int j = 0; j < x.k; ++j)
        if (x.q[j] != y.q[j]) return false;
    return true;
}

// Product (application order) of ops[src[s..e)], all on the same targets.
LOp local_product(const std::vector<LOp> &ops, const std::vector<int> &src, size_t s, size_t e)
{
    const LOp &a = ops[src[s]];
    const int D = 1 << (2 * a.k);
    LOp out;
    out.k = a.k;
    for (int j = 0; j < a.k; ++j) out.q[j] = a.q[j];
    bool all_diag = true;
    for (size_t i = s; i < e; ++i) all_diag &= ops[src[i]].diag;
    if (all_diag) {
        out.diag = true;
        out.D.assign(D, cd(1));
        for (size_t i = s; i < e; ++i)
            for (int x = 0; x < D; ++x) out.D[x] *= ops[src[i]].D[x];
        return out;
    }
    std::vector<cd> M(size_t(D) * D, cd(0)), T(size_t(D) * D);
    for (int x = 0; x < D; ++x) M[size_t(x) * D + x] = 1.0;
    for (size_t i = s; i < e; ++i) {
        const LOp &o = ops[src[i]];
        std::fill(T.begin(), T.end(), cd(0));
        for (int r = 0; r < D; ++r)
            if (o.diag) {
                for (int c = 0; c < D; ++c) T[size_t(r) * D + c] = o.D[r] * M[size_t(r) * D + c];
            } else {
                for (int k = 0; k < D; ++k) {
                    const cd v = o.S[size_t(r) * D + k];
                    if (is_zero(v)) continue;
                    for (int c = 0; c < D; ++c) T[size_t(r) * D + c] += v * M[size_t(k) * D + c];
                }
            }
        M.swap(T);
    }
    out.S = std::move(M);
    return out;
}

}  // namespace

int recompute_mats(int n, const HostPlan &plan, const std::vector<LOp> &ops, std::vector<cd> &mats)
{
    mats.resize(plan.mats.size());
    std::fill(mats.begin(), mats.end(), cd(0));
    if (plan.recipes.size() != plan.ops.size())
        return fail(VQD_E_STATE, "plan has no coefficient recipes");
    for (const Recipe &r : plan.recipes) {
        for (int s : r.src)
            if (s < 0 || s >= (int)ops.size()) return fail(VQD_E_ARG, "recipe refers to a missing op");
        if (r.rt) {
            for (const RtPart &pt : r.rt_parts)
                if (!ops[pt.src].diag)
                    return fail(VQD_E_ARG, "op structure differs from the template (diagonal expected)");
            thread_local std::vector<cd> table;
            rt_table(r.mode, r.rt_union, r.rt_parts, ops, table);
            if (r.real && !all_real(table))
                return fail(VQD_E_ARG, "op structure differs from the template (complex diagonal)");
            for (size_t i = 0; i < table.size(); ++i) mats[r.mat_off + i] = table[i];
            continue;
        }
        if (r.mode >= 100) return fail(VQD_E_ARG, "wide unitary blocks cannot be recomputed");
        // product in application order; a run of ops on the same targets is
        // first multiplied in its own 4^k space, then embedded once
        Mat16 m{};
        bool first = true;
        for (size_t s = 0; s < r.src.size();) {
            const LOp &a = ops[r.src[s]];
            size_t e = s + 1;
            while (e < r.src.size() && same_targets(ops[r.src[e]], a)) ++e;
            uint32_t sup = 0;
            Mat16 emb = (e - s == 1) ? embed(a, n, r.reg_gpos, sup)
                                     : embed(local_product(ops, r.src, s, e), n, r.reg_gpos, sup);
            m = first ? emb : mul(emb, m);
            first = false;
            s = e;
        }
        if (first)
            for (int e = 0; e < 16; ++e) m[e * 16 + e] = 1.0;
        // the new coefficients must fit the form chosen for the template's
        // (per-thread scratch: this runs once per recipe of every instance)
        thread_local std::vector<cd> data, sub;
        thread_local std::vector<int> fl;
        data.clear();
        if (r.kind == KOP_DIAG) {
            data.resize(16);
            for (int i = 0; i < 16; ++i)
                for (int j = 0; j < 16; ++j)
                    if (i != j && !is_zero(m[i * 16 + j]))
                        return fail(VQD_E_ARG, "op structure differs from the template (not diagonal)");
            for (int e = 0; e < 16; ++e) data[e] = m[e * 16 + e];
        } else {
            if (!restrict_to(m, (int)r.mask, sub))
                return fail(VQD_E_ARG, "op structure differs from the template");
            const int dim = 1 << popc(r.mask);
            if (r.kind == KOP_PTM) {
                thread_local std::vector<double> rows;
                if (!ptm_of(sub, rows))
                    return fail(VQD_E_ARG, "op structure differs from the template (Pauli transfer form)");
                data.assign(rows.begin(), rows.end());
            } else if (r.kind == KOP_MAT) {
                data.resize(size_t(dim) * dim);
                for (int j = 0; j < dim; ++j)
                    for (int i = 0; i < dim; ++i) data[j * dim + i] = sub[i * dim + j];
            } else {
                fl = local_flips((int)r.mask);
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j)
                        if (!is_zero(sub[i * dim + j]) && std::find(fl.begin(), fl.end(), i ^ j) == fl.end())
                            return fail(VQD_E_ARG, "op structure differs from the template (flip pattern)");
                data.resize(fl.size() * dim);
                for (size_t x = 0; x < fl.size(); ++x)
                    for (int i = 0; i < dim; ++i) data[x * dim + i] = sub[i * dim + (i ^ fl[x])];
            }
        }
        if (r.real && !all_real(data))
            return fail(VQD_E_ARG, "op structure differs from the template (complex coefficients)");
        // pool layout: complex entries as they are, real ones two per entry
        if (r.real) {
            for (size_t i = 0; i < data.size(); ++i) {
                cd &o = mats[r.mat_off + i / 2];
                if (i & 1) o.imag(data[i].real());
                else o = cd(data[i].real(), 0.0);
            }
        } else {
            for (size_t i = 0; i < data.size(); ++i) mats[r.mat_off + i] = data[i];
        }
    }
    return VQD_OK;
}

int upload_plan(const HostPlan &plan, DevProgram &dev, hipStream_t stream)
{
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t b_pass = align(plan.passes.size() * sizeof(KPass));
    const size_t b_phase = align(plan.phases.size() * sizeof(KPhase));
    const size_t b_ops = align(plan.ops.size() * sizeof(KOp));
    const size_t b_mats = align(plan.mats.size() * sizeof(double2));
    const size_t total = b_pass + b_phase + b_ops + b_mats + 256;
    if (dev.bytes < total) {
        if (dev.buf) {
            VQD_HIP(hipStreamSynchronize(stream));
            (void)hipFree(dev.buf);
        }
        dev.buf = nullptr;
        dev.bytes = 0;
        if (hipMalloc(&dev.buf, total) != hipSuccess)
            return fail(VQD_E_NOMEM, "descriptor allocation failed");
        dev.bytes = total;
    }
    // staging copy (not zero-filled: every byte up to `off` is written below)
    std::unique_ptr<unsigned char[]> host_buf(new (std::nothrow) unsigned char[total]);
    if (!host_buf) return fail(VQD_E_NOMEM, "descriptor staging allocation failed");
    unsigned char *const host = host_buf.get();
    const size_t mats_bytes = plan.mats.size() * sizeof(double2);
    std::memset(host, 0, b_pass + b_phase + b_ops);             // descriptor sections and their padding
    std::memset(host + b_pass + b_phase + b_ops + mats_bytes, 0, b_mats - mats_bytes);
    size_t off = 0;
    std::memcpy(host + off, plan.passes.data(), plan.passes.size() * sizeof(KPass));
    dev.passes = reinterpret_cast<KPass *>((char *)dev.buf + off);
    off += b_pass;
    std::memcpy(host + off, plan.phases.data(), plan.phases.size() * sizeof(KPhase));
    dev.phases = reinterpret_cast<KPhase *>((char *)dev.buf + off);
    off += b_phase;
    std::memcpy(host + off, plan.ops.data(), plan.ops.size() * sizeof(KOp));
    dev.ops = reinterpret_cast<KOp *>((char *)dev.buf + off);
    off += b_ops;
    // std::complex<double> is laid out as (re, im), as double2
    static_assert(sizeof(cd) == sizeof(double2), "complex layout");
    std::memcpy(host + off, plan.mats.data(), mats_bytes);
    dev.mats = reinterpret_cast<double2 *>((char *)dev.buf + off);
    off += b_mats;
    // ordered on the stream after earlier work that read the old descriptors;
    // the synchronisation keeps the staging vector alive until the copy ends
    VQD_HIP(hipMemcpyAsync(dev.buf, host, off, hipMemcpyHostToDevice, stream));
    VQD_HIP(hipStreamSynchronize(stream));
    return VQD_OK;
}

void free_dev_program(DevProgram &dev)
{
    if (dev.buf) (void)hipFree(dev.buf);
    dev = DevProgram{};
}

}  // namespace vqd
