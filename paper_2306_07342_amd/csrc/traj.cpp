// Monte Carlo trajectory mode (declarations and contract in include/vqd.h):
// op programs on a state vector, their phase plan and the batched launch.
//
// Planning.  A phase fixes four qubits as the register bits of every thread;
// an op may run in a phase when its qubits are register qubits (diagonal
// gates may run anywhere).  Ops are scheduled in order, except that an op
// may be taken before earlier pending ops it commutes with: ops on disjoint
// qubits, of which at most one is a channel (gates are unitary, so moving one
// past a channel on other qubits leaves that channel's weights unchanged).
// Channels therefore keep their relative order and meet their uniforms in
// channel order.  Consecutive gates of a phase whose qubit sets nest are
// multiplied into one matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vqd_internal.h"

namespace vqd {
namespace {

constexpr int kWindow = 48;          // pending ops a phase may draw from
constexpr double kUnitaryTol = 1e-10;
constexpr double kMixedTol = 1e-12;

struct TIn {
    int k = 0;
    int q[4] = {0, 0, 0, 0};
    bool chan = false;
    bool diag = false;                       // gate with a diagonal matrix
    std::vector<cd> M;                       // gate: 2^k x 2^k row-major
    std::vector<std::vector<cd>> K;          // channel: Kraus operators, row-major
};

// A gate or channel of a phase, before encoding.
struct POp {
    bool chan = false;
    bool diag = false;
    std::vector<int> qs;                     // matrix bit j acts on qubit qs[j]
    std::vector<cd> M;
    const TIn *src = nullptr;
    uint32_t chan_idx = 0;
};

// Row-major product A B of D x D matrices.
std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, int D)
{
    std::vector<cd> C(size_t(D) * D, cd(0));
    for (int r = 0; r < D; ++r)
        for (int k = 0; k < D; ++k) {
            const cd a = A[size_t(r) * D + k];
            if (a == cd(0)) continue;
            for (int c = 0; c < D; ++c) C[size_t(r) * D + c] += a * B[size_t(k) * D + c];
        }
    return C;
}

// M (bit j on qubit mq[j]) as a matrix on the qubits uq (bit j on uq[j]),
// identity on the qubits of uq that M does not act on.
std::vector<cd> embed(const std::vector<cd> &M, const std::vector<int> &mq, const std::vector<int> &uq)
{
    const int mk = (int)mq.size(), d = 1 << mk, D = 1 << (int)uq.size();
    std::vector<int> pos(mk);
    int mbits = 0;
    for (int j = 0; j < mk; ++j) {
        pos[j] = int(std::find(uq.begin(), uq.end(), mq[j]) - uq.begin());
        mbits |= 1 << pos[j];
    }
    std::vector<cd> E(size_t(D) * D, cd(0));
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            if ((r & ~mbits) != (c & ~mbits)) continue;
            int rm = 0, cm = 0;
            for (int j = 0; j < mk; ++j) {
                rm |= ((r >> pos[j]) & 1) << j;
                cm |= ((c >> pos[j]) & 1) << j;
            }
            E[size_t(r) * D + c] = M[size_t(rm) * d + cm];
        }
    return E;
}

bool is_diagonal(const std::vector<cd> &M, int d)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && M[size_t(r) * d + c] != cd(0)) return false;
    return true;
}

bool is_unitary(const std::vector<cd> &U, int d)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            cd s(0);
            for (int k = 0; k < d; ++k) s += std::conj(U[size_t(k) * d + r]) * U[size_t(k) * d + c];
            if (std::abs(s - cd(r == c ? 1.0 : 0.0)) > kUnitaryTol) return false;
        }
    return true;
}

// K^dagger K (row-major).
std::vector<cd> gram(const std::vector<cd> &K, int d)
{
    std::vector<cd> G(size_t(d) * d, cd(0));
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            cd s(0);
            for (int k = 0; k < d; ++k) s += std::conj(K[size_t(k) * d + r]) * K[size_t(k) * d + c];
            G[size_t(r) * d + c] = s;
        }
    return G;
}

bool contains(const std::vector<int> &big, const std::vector<int> &small)
{
    for (int x : small)
        if (std::find(big.begin(), big.end(), x) == big.end()) return false;
    return true;
}

}  // namespace
}  // namespace vqd

using vqd::cd;

struct vqd_traj {
    int n = 0;
    int n_eff = 4;
    std::vector<vqd::TIn> ops;
    int n_channels = 0;
    // plan
    std::vector<vqd::TPhase> phases;
    std::vector<vqd::TOp> kops;
    std::vector<cd> pool;
    double fma_per_amp = 0.0;
    int n_mixed = 0, n_general = 0;
    // device image
    void *buf = nullptr;
    size_t bytes = 0;
    vqd::TPhase *d_phases = nullptr;
    vqd::TOp *d_ops = nullptr;
    double2 *d_pool = nullptr;
    bool compiled = false;
    int device = -1;
};

namespace vqd {
namespace {

int traj_push(vqd_traj *t, TIn op)
{
    try {
        if (op.chan) ++t->n_channels;
        t->ops.push_back(std::move(op));
    } catch (...) {
        return fail(VQD_E_NOMEM, "out of host memory");
    }
    t->compiled = false;
    return VQD_OK;
}

int make_gate(int k, const int *targets, std::vector<cd> U, TIn &op)
{
    const int d = 1 << k;
    if (!is_unitary(U, d)) return fail(VQD_E_ARG, "gate matrix is not unitary");
    op.k = k;
    for (int j = 0; j < k; ++j) op.q[j] = targets[j];
    op.chan = false;
    op.diag = is_diagonal(U, d);
    op.M = std::move(U);
    return VQD_OK;
}

// Append the coefficients of M (bit j on qubit qs[j]) for the register
// layout R: bits reordered to ascending register bit, column-major.  Returns
// the register mask.
uint32_t put_matrix(std::vector<cd> &pool, const std::vector<cd> &M, const std::vector<int> &qs, const int *R,
                    bool col_major)
{
    std::vector<int> order;
    uint32_t mask = 0;
    for (int b = 0; b < 4; ++b)
        if (std::find(qs.begin(), qs.end(), R[b]) != qs.end()) {
            order.push_back(R[b]);
            mask |= 1u << b;
        }
    const std::vector<cd> P = embed(M, qs, order);
    const int d = 1 << (int)order.size();
    for (int x = 0; x < d; ++x)
        for (int y = 0; y < d; ++y) pool.push_back(col_major ? P[size_t(y) * d + x] : P[size_t(x) * d + y]);
    return mask;
}

// Encode the ops of one phase with register qubits R.
int encode_phase(vqd_traj *t, const int *R, const std::vector<POp> &ops)
{
    const size_t first_k = t->kops.size();
    for (const POp &o : ops) {
        TOp k{};
        const int nq = (int)o.qs.size(), d = 1 << nq;
        if (!o.chan) {
            if (o.diag && nq <= 2) {
                // where the qubits are: register bit or -1 (a thread qubit)
                int rb[2] = {-1, -1};
                for (int j = 0; j < nq; ++j)
                    for (int b = 0; b < 4; ++b)
                        if (R[b] == o.qs[j]) rb[j] = b;
                const int n_reg = (rb[0] >= 0) + (nq > 1 && rb[1] >= 0);
                bool real = true;
                for (int x = 0; x < d; ++x) real = real && o.M[size_t(x) * d + x].imag() == 0.0;
                k.mat = (uint32_t)t->pool.size();
                k.real = real ? 1u : 0u;
                if (n_reg == nq) {
                    // factor of register slot e: matrix index bit j = slot bit rb[j]
                    k.kind = TOP_DREG;
                    for (int e = 0; e < 16; ++e) {
                        int x = 0;
                        for (int j = 0; j < nq; ++j) x |= ((e >> rb[j]) & 1) << j;
                        t->pool.push_back(o.M[size_t(x) * d + x]);
                    }
                } else if (n_reg == 0) {
                    k.kind = TOP_DTHR;
                    k.nd = (uint32_t)nq;
                    k.dq[0] = (uint32_t)o.qs[0];
                    k.dq[1] = nq > 1 ? (uint32_t)o.qs[1] : 0u;
                    for (int x = 0; x < d; ++x) t->pool.push_back(o.M[size_t(x) * d + x]);
                } else {
                    // one register qubit jr, one thread qubit jt
                    const int jr = rb[0] >= 0 ? 0 : 1, jt = 1 - jr;
                    k.kind = TOP_DMIX;
                    k.mask = 1u << rb[jr];
                    k.dq[0] = (uint32_t)o.qs[jt];
                    for (int tb = 0; tb < 2; ++tb)
                        for (int r = 0; r < 2; ++r) {
                            const int x = (tb << jt) | (r << jr);
                            t->pool.push_back(o.M[size_t(x) * d + x]);
                        }
                }
                t->fma_per_amp += real ? 2.0 : 4.0;
            } else {
                bool real = true;
                for (const cd &z : o.M) real = real && z.imag() == 0.0;
                std::vector<cd> tmp;
                k.kind = TOP_MAT;
                k.mask = put_matrix(tmp, o.M, o.qs, R, true);
                k.mat = (uint32_t)t->pool.size();
                k.real = real ? 1u : 0u;
                if (real) {
                    for (size_t i = 0; i < tmp.size(); i += 2)
                        t->pool.push_back(cd(tmp[i].real(), i + 1 < tmp.size() ? tmp[i + 1].real() : 0.0));
                } else {
                    t->pool.insert(t->pool.end(), tmp.begin(), tmp.end());
                }
                t->fma_per_amp += (real ? 2.0 : 4.0) * d;
            }
        } else {
            const std::vector<std::vector<cd>> &Ks = o.src->K;
            // mixed unitary: every K^dagger K is a multiple q of the identity
            bool mixed = true;
            std::vector<double> q;
            std::vector<std::vector<cd>> Gs;
            for (const auto &K : Ks) {
                std::vector<cd> G = gram(K, d);
                double tr = 0.0;
                for (int x = 0; x < d; ++x) tr += G[size_t(x) * d + x].real();
                const double qi = tr / d;
                for (int x = 0; x < d && mixed; ++x)
                    for (int y = 0; y < d; ++y)
                        if (std::abs(G[size_t(x) * d + y] - cd(x == y ? qi : 0.0)) > kMixedTol) {
                            mixed = false;
                            break;
                        }
                q.push_back(qi);
                Gs.push_back(std::move(G));
            }
            k.chan = o.chan_idx;
            k.mat = (uint32_t)t->pool.size();
            // operators that are diagonal (and real) take the kernel's
            // per-slot path when drawn; channels are counted at the cost of
            // their most probable operator (for a general channel: largest
            // Tr(K^dagger K), its weight on the maximally mixed state)
            auto diag_of = [&](const std::vector<cd> &K, bool &real) {
                real = true;
                for (int x = 0; x < d; ++x)
                    for (int y = 0; y < d; ++y) {
                        const cd z = K[size_t(x) * d + y];
                        if (x != y && z != cd(0)) return false;
                        if (x == y) real = real && z.imag() == 0.0;
                    }
                return true;
            };
            auto op_cost = [&](const std::vector<cd> &K) {
                bool real = false;
                return diag_of(K, real) ? (real ? 2.0 : 4.0) : 4.0 * d;
            };
            if (mixed) {
                k.kind = TOP_MIX;
                std::vector<size_t> keep;
                for (size_t i = 0; i < Ks.size(); ++i)
                    if (q[i] > 0.0) keep.push_back(i);
                if (keep.empty()) return fail(VQD_E_ARG, "channel with all-zero Kraus operators");
                k.nk = (uint32_t)keep.size();
                // (running sum of the weights in index order, weight): the
                // kernel draws by comparing u W with the running sums
                double cum = 0.0;
                for (size_t i : keep) {
                    cum += q[i];
                    t->pool.push_back(cd(cum, q[i]));
                }
                size_t mode = keep[0];
                std::vector<size_t> at;              // pool offset of each operator
                for (size_t j = 0; j < keep.size(); ++j) {
                    const size_t i = keep[j];
                    std::vector<cd> U = Ks[i];
                    const double s = 1.0 / std::sqrt(q[i]);
                    for (cd &z : U) z *= s;
                    bool real = false;
                    if (diag_of(U, real)) {
                        k.dmask |= 1u << j;
                        if (real) k.rmask |= 1u << j;
                    }
                    if (q[i] > q[mode]) mode = i;
                    at.push_back(t->pool.size());
                    k.mask = put_matrix(t->pool, U, o.qs, R, true);
                }
                bool first_identity = true;         // operator 0 stored exactly as the identity
                for (int y = 0; y < d; ++y)
                    for (int x = 0; x < d; ++x)
                        first_identity = first_identity && t->pool[at[0] + size_t(y) * d + x] == cd(x == y ? 1.0 : 0.0);
                if (d == 2 && k.nk == 2 && k.rmask == 3u) {
                    k.inl = 1;
                    k.cf[0] = t->pool[k.mat].real();
                    k.cf[1] = t->pool[k.mat + 1].real();
                    for (int j = 0; j < 2; ++j) {
                        k.cf[2 + 2 * j] = t->pool[at[j]].real();         // column-major (0, 0)
                        k.cf[3 + 2 * j] = t->pool[at[j] + 3].real();     // (1, 1)
                    }
                } else if (k.nk >= 2 && first_identity) {
                    // the common draw, operator 0 = the identity, needs only
                    // the first running sum and the total
                    k.inl = 2;
                    k.cf[0] = t->pool[k.mat].real();
                    k.cf[1] = t->pool[k.mat + k.nk - 1].real();
                }
                ++t->n_mixed;
                std::vector<cd> Um = Ks[mode];
                for (cd &z : Um) z /= std::sqrt(q[mode]);
                t->fma_per_amp += op_cost(Um);
            } else {
                k.kind = TOP_KRAUS;
                k.nk = (uint32_t)Ks.size();
                k.gdiag = 1;
                std::vector<size_t> gat, kat;        // pool offsets of the G_i and K_i
                for (const auto &G : Gs) {
                    bool real = false;
                    if (!diag_of(G, real)) k.gdiag = 0;
                    gat.push_back(t->pool.size());
                    put_matrix(t->pool, G, o.qs, R, false);
                }
                size_t mode = 0;
                for (size_t i = 0; i < Ks.size(); ++i) {
                    bool real = false;
                    if (diag_of(Ks[i], real)) {
                        k.dmask |= 1u << i;
                        if (real) k.rmask |= 1u << i;
                    }
                    if (q[i] > q[mode]) mode = i;
                    kat.push_back(t->pool.size());
                    k.mask = put_matrix(t->pool, Ks[i], o.qs, R, true);
                }
                if (d == 2 && k.nk == 2 && k.gdiag && (k.rmask & 1u)) {
                    k.inl = 1;
                    for (int i = 0; i < 2; ++i) {
                        k.cf[2 * i] = t->pool[gat[i]].real();             // (0, 0)
                        k.cf[2 * i + 1] = t->pool[gat[i] + 3].real();     // (1, 1)
                    }
                    k.cf[4] = t->pool[kat[0]].real();
                    k.cf[5] = t->pool[kat[0] + 3].real();
                }
                ++t->n_general;
                // drawn operator, its scaling, and this thread's part of rho_T
                t->fma_per_amp += op_cost(Ks[mode]) + 2.0 + (k.gdiag ? 2.0 : 2.0 * d);
            }
        }
        // a register diagonal right after another one: one set of 16
        // factors, their products (diagonal factors commute)
        if (k.kind == TOP_DREG && t->kops.size() > first_k && t->kops.back().kind == TOP_DREG &&
            k.mat + kSlots == t->pool.size()) {
            TOp &p = t->kops.back();
            for (int e = 0; e < kSlots; ++e) t->pool[p.mat + e] *= t->pool[k.mat + e];
            t->pool.resize(k.mat);
            p.real = (p.real && k.real) ? 1u : 0u;
            t->fma_per_amp -= k.real ? 2.0 : 4.0;
            continue;
        }
        // a register diagonal and a one-register, one-thread-qubit diagonal
        // next to each other (either order): one op, one descriptor and one
        // coefficient block
        if (t->kops.size() > first_k && !t->kops.back().inl) {
            TOp &p = t->kops.back();
            const bool reg_then_mix = p.kind == TOP_DREG && k.kind == TOP_DMIX && k.mat + 4 == t->pool.size() &&
                                      p.mat + kSlots == k.mat;
            const bool mix_then_reg = p.kind == TOP_DMIX && k.kind == TOP_DREG &&
                                      k.mat + kSlots == t->pool.size() && p.mat + 4 == k.mat;
            // one-qubit gates in a row on register bits (each 2x2, complex,
            // column-major), up to four
            auto one_bit = [](const TOp &o) {
                return o.kind == TOP_MAT && (o.mask == 1u || o.mask == 2u || o.mask == 4u || o.mask == 8u);
            };
            auto coefs = [&](const TOp &o, std::vector<cd> &c) {
                if (o.real) {
                    for (int i = 0; i < 2; ++i) {
                        c.push_back(cd(t->pool[o.mat + i].real(), 0.0));
                        c.push_back(cd(t->pool[o.mat + i].imag(), 0.0));
                    }
                } else {
                    for (int i = 0; i < 4; ++i) c.push_back(t->pool[o.mat + i]);
                }
            };
            auto bit_of = [](uint32_t m) { return (uint32_t)__builtin_ctz(m); };
            const bool p_mats = p.kind == TOP_MATS && p.nd < 4u;
            if (one_bit(k) && (one_bit(p) || p_mats) && k.mat + (k.real ? 2u : 4u) == t->pool.size()) {
                std::vector<cd> block;
                if (p_mats) {
                    for (uint32_t i = 0; i < 4u * p.nd; ++i) block.push_back(t->pool[p.mat + i]);
                } else {
                    coefs(p, block);
                    p.dmask = bit_of(p.mask);
                    p.nd = 1;
                }
                coefs(k, block);
                if (p.mat + (p_mats ? 4u * p.nd : (p.real ? 2u : 4u)) == k.mat) {
                    t->pool.resize(p.mat);
                    t->pool.insert(t->pool.end(), block.begin(), block.end());
                    p.dmask |= bit_of(k.mask) << (2u * p.nd);
                    ++p.nd;
                    p.kind = TOP_MATS;
                    p.real = 0;
                    continue;
                }
                if (!p_mats) {   // not adjacent in the pool: leave both as they are
                    p.nd = 0;
                    p.dmask = 0;
                }
            }
            if (p.kind == TOP_DMIX && k.kind == TOP_DMIX && p.mat + 4 == k.mat && k.mat + 4 == t->pool.size()) {
                p.kind = TOP_DMIX2;
                p.dmask = k.mask;
                p.dq[1] = k.dq[0];
                p.real = (p.real && k.real) ? 1u : 0u;
                continue;
            }
            if (reg_then_mix || mix_then_reg) {
                std::vector<cd> block(kSlots + 4);
                const size_t reg_at = reg_then_mix ? p.mat : k.mat, mix_at = reg_then_mix ? k.mat : p.mat;
                for (int e = 0; e < kSlots; ++e) block[e] = t->pool[reg_at + e];
                for (int j = 0; j < 4; ++j) block[kSlots + j] = t->pool[mix_at + j];
                std::copy(block.begin(), block.end(), t->pool.begin() + p.mat);
                const TOp &mix = reg_then_mix ? k : p;
                const uint32_t mask = mix.mask, dq0 = mix.dq[0];
                p.kind = TOP_DRM;
                p.mask = mask;
                p.dq[0] = dq0;
                p.real = (p.real && k.real) ? 1u : 0u;
                continue;
            }
        }
        t->kops.push_back(k);
    }
    return VQD_OK;
}

// Runs of one-qubit channels with inline coefficients (TOp::grp).  A
// mixed-unitary member must leave every population as it is (diagonal
// entries of magnitude 1, up to the rounding of the stored unitary's
// normalisation), so that the damping members' weights can all be formed
// from the run's input state; a damping member must be trace preserving.
constexpr double kUnitTol = 1e-15;

void mark_groups(std::vector<TOp> &kops, uint32_t begin, uint32_t end)
{
    auto member = [&](const TOp &k) {
        if (k.inl != 1u) return false;
        // damping: trace preserving (G0 + G1 = I), so that a run's draws
        // need only the running sums of the no-jump weights
        if (k.kind == TOP_KRAUS)
            return std::abs(k.cf[0] + k.cf[2] - 1.0) <= kUnitTol && std::abs(k.cf[1] + k.cf[3] - 1.0) <= kUnitTol;
        if (k.kind != TOP_MIX) return false;
        for (int j = 2; j < 6; ++j)
            if (std::abs(std::abs(k.cf[j]) - 1.0) > kUnitTol) return false;
        return true;
    };
    uint32_t i = begin;
    while (i < end) {
        if (!member(kops[i])) {
            ++i;
            continue;
        }
        uint32_t j = i, kraus = 0;
        while (j < end && j - i < kTrajGroupMax && member(kops[j])) {
            const bool damp = kops[j].kind == TOP_KRAUS;
            if (damp && kraus == kTrajGroupKraus) break;
            kraus += damp ? 1u : 0u;
            ++j;
        }
        if (kraus >= 2) kops[i].grp = j - i;
        i = j;
    }
}

int plan(vqd_traj *t)
{
    t->phases.clear();
    t->kops.clear();
    t->pool.clear();
    t->fma_per_amp = 0.0;
    t->n_mixed = t->n_general = 0;
    const int ne = t->n_eff;
    const std::vector<TIn> &ops = t->ops;
    std::vector<int> chan_idx(ops.size(), 0);
    {
        int c = 0;
        for (size_t i = 0; i < ops.size(); ++i)
            if (ops[i].chan) chan_idx[i] = c++;
    }
    auto commute = [&](const TIn &a, const TIn &b) {
        if (a.chan && b.chan) return false;
        for (int i = 0; i < a.k; ++i)
            for (int j = 0; j < b.k; ++j)
                if (a.q[i] == b.q[j]) return false;
        return true;
    };
    std::vector<int> pending(ops.size());
    for (size_t i = 0; i < ops.size(); ++i) pending[i] = (int)i;
    size_t head = 0;                       // pending[head..] are unscheduled
    auto movable = [&](size_t p) {
        for (size_t e = head; e < p; ++e)
            if (!commute(ops[pending[e]], ops[pending[p]])) return false;
        return true;
    };
    auto needs_regs = [&](const TIn &o) { return o.chan || !o.diag || o.k > 2; };
    uint32_t expect_chan = 0;
    while (head < pending.size()) {
        // the register qubits and the phase's ops together: walk the pending
        // ops in order and take each op that commutes with every earlier
        // pending op and whose qubits fit the register set (which grows up
        // to four qubits), until a walk takes nothing
        std::vector<int> R;
        std::vector<POp> taken;
        bool progress = true;
        while (progress) {
            progress = false;
            const size_t lim = std::min(pending.size(), head + kWindow);
            for (size_t p = head; p < lim; ++p) {
                const TIn &o = ops[pending[p]];
                if (!movable(p)) continue;
                if (needs_regs(o)) {
                    std::vector<int> u = R;
                    for (int j = 0; j < o.k; ++j)
                        if (std::find(u.begin(), u.end(), o.q[j]) == u.end()) u.push_back(o.q[j]);
                    if (u.size() > 4) continue;
                    R = u;
                }
                POp po;
                po.chan = o.chan;
                po.diag = o.diag;
                po.qs.assign(o.q, o.q + o.k);
                po.M = o.M;
                po.src = &o;
                po.chan_idx = (uint32_t)chan_idx[pending[p]];
                if (o.chan && po.chan_idx != expect_chan++)
                    return fail(VQD_E_STATE, "internal: channels out of order");
                taken.push_back(std::move(po));
                // remove pending[p] keeping the order of the rest
                std::rotate(pending.begin() + head, pending.begin() + p, pending.begin() + p + 1);
                ++head;
                progress = true;
            }
        }
        for (int q = 0; q < ne && R.size() < 4; ++q)
            if (std::find(R.begin(), R.end(), q) == R.end()) R.push_back(q);
        std::sort(R.begin(), R.end());
        if (taken.empty()) return fail(VQD_E_STATE, "internal: planner made no progress");
        // fuse consecutive gates whose qubit sets nest
        std::vector<POp> fused;
        for (POp &o : taken) {
            if (!o.chan && !fused.empty() && !fused.back().chan) {
                POp &L = fused.back();
                const bool o_in_L = contains(L.qs, o.qs), L_in_o = contains(o.qs, L.qs);
                if (o_in_L || L_in_o) {
                    const std::vector<int> U = o_in_L ? L.qs : o.qs;
                    const bool diag = L.diag && o.diag;
                    bool in_regs = true;
                    for (int x : U) in_regs = in_regs && std::find(R.begin(), R.end(), x) != R.end();
                    if ((diag && U.size() <= 2) || in_regs) {
                        const int D = 1 << (int)U.size();
                        L.M = matmul(embed(o.M, o.qs, U), embed(L.M, L.qs, U), D);
                        L.qs = U;
                        L.diag = diag;
                        continue;
                    }
                }
            }
            fused.push_back(std::move(o));
        }
        TPhase ph{};
        ph.op_begin = (uint32_t)t->kops.size();
        for (int b = 0; b < 4; ++b) ph.reg_q[b] = (uint32_t)R[b];
        // thread qubits: the first three (lane bits 0-2) at index positions of
        // residue 0, 1, 2 mod 3 where possible, which the LDS index swizzle
        // spreads over distinct 16-byte bank groups; the rest ascending
        std::vector<int> rest;
        for (int q = 0; q < ne; ++q)
            if (std::find(R.begin(), R.end(), q) == R.end()) rest.push_back(q);
        int ti = 0;
        for (int i = 0; i < 3 && !rest.empty(); ++i) {
            auto it = std::find_if(rest.begin(), rest.end(), [&](int q) { return q % 3 == i && q < 12; });
            if (it == rest.end()) it = rest.begin();
            ph.thr_q[ti++] = (uint32_t)*it;
            rest.erase(it);
        }
        for (int q : rest) ph.thr_q[ti++] = (uint32_t)q;
        if (int rc = encode_phase(t, R.data(), fused)) return rc;
        ph.op_end = (uint32_t)t->kops.size();
        mark_groups(t->kops, ph.op_begin, ph.op_end);
        for (uint32_t i = ph.op_begin; i < ph.op_end; ++i)
            if (t->kops[i].kind == TOP_KRAUS) ph.flags |= kTPhaseReduces;
        t->phases.push_back(ph);
    }
    if (t->phases.empty()) {
        // no op at all: one empty phase still initialises and reads out
        TPhase ph{};
        for (int b = 0; b < 4; ++b) ph.reg_q[b] = (uint32_t)b;
        for (int q = 4; q < ne; ++q) ph.thr_q[q - 4] = (uint32_t)q;
        t->phases.push_back(ph);
    }
    // per-slot LDS index parts (the swizzle is xor-linear in the index bits)
    for (TPhase &ph : t->phases)
        for (int e = 0; e < kSlots; ++e) {
            uint32_t l = 0;
            for (int b = 0; b < 4; ++b)
                if (e >> b & 1) l |= 1u << (ph.reg_q[b] & 31u);
            ph.lds_slot[e] = lds_swizzle(l);
        }
    // the kernels may read up to 16 operators of 16 entries past an op's data
    t->pool.resize(t->pool.size() + 256, cd(0));
    return VQD_OK;
}

int upload(vqd_traj *t)
{
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t b_ph = align(t->phases.size() * sizeof(TPhase));
    const size_t b_op = align(std::max<size_t>(1, t->kops.size()) * sizeof(TOp));
    const size_t b_pool = align(t->pool.size() * sizeof(double2));
    const size_t total = b_ph + b_op + b_pool;
    if (t->buf) {
        (void)hipFree(t->buf);
        t->buf = nullptr;
        t->bytes = 0;
    }
    if (hipMalloc(&t->buf, total) != hipSuccess) return fail(VQD_E_NOMEM, "descriptor allocation failed");
    t->bytes = total;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data(), t->phases.data(), t->phases.size() * sizeof(TPhase));
    if (!t->kops.empty()) std::memcpy(host.data() + b_ph, t->kops.data(), t->kops.size() * sizeof(TOp));
    for (size_t i = 0; i < t->pool.size(); ++i) {
        const double v[2] = {t->pool[i].real(), t->pool[i].imag()};
        std::memcpy(host.data() + b_ph + b_op + i * sizeof(double2), v, sizeof(v));
    }
    VQD_HIP(hipMemcpy(t->buf, host.data(), total, hipMemcpyHostToDevice));
    t->d_phases = reinterpret_cast<TPhase *>(t->buf);
    t->d_ops = reinterpret_cast<TOp *>((char *)t->buf + b_ph);
    t->d_pool = reinterpret_cast<double2 *>((char *)t->buf + b_ph + b_op);
    return VQD_OK;
}

}  // namespace
}  // namespace vqd

using namespace vqd;

extern "C" {

int vqd_traj_create(int n, vqd_traj **out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > kTrajMaxQubits)
        return fail(VQD_E_SIZE, "trajectories need n in [1, " + std::to_string(kTrajMaxQubits) + "]");
    vqd_traj *t = new (std::nothrow) vqd_traj;
    if (!t) return fail(VQD_E_NOMEM, "out of host memory");
    t->n = n;
    t->n_eff = std::max(n, 4);
    *out = t;
    return VQD_OK;
}

int vqd_traj_destroy(vqd_traj *t)
{
    clear_error();
    if (!t) return VQD_OK;
    if (t->buf) (void)hipFree(t->buf);
    delete t;
    return VQD_OK;
}

int vqd_traj_add_named(vqd_traj *t, int kind, const int *targets, const double *params)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    int nq = 0, np = 0;
    if (kind_arity(kind, &nq, &np) != 0) return fail(VQD_E_ARG, "unknown kind " + std::to_string(kind));
    if (int rc = check_targets(t->n, nq, targets)) return rc;
    if (np > 0 && !params) return fail(VQD_E_ARG, "null params");
    TIn op;
    if (kind_is_channel(kind)) {
        int k = 0;
        if (int rc = kind_kraus(kind, params, op.K, k)) return rc;
        op.k = k;
        for (int j = 0; j < k; ++j) op.q[j] = targets[j];
        op.chan = true;
    } else {
        std::vector<cd> U;
        int k = 0;
        if (int rc = kind_matrix(kind, params, U, k)) return rc;
        if (int rc = make_gate(k, targets, std::move(U), op)) return rc;
    }
    return traj_push(t, std::move(op));
}

int vqd_traj_add_named_many(vqd_traj *t, int count, const int *kinds, const int *targets, const double *params)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    if (count < 0 || (count > 0 && (!kinds || !targets || !params))) return fail(VQD_E_ARG, "bad arrays");
    const size_t before = t->ops.size();
    const int ch_before = t->n_channels;
    for (int i = 0; i < count; ++i) {
        const int rc = vqd_traj_add_named(t, kinds[i], targets + 4 * (size_t)i, params + 4 * (size_t)i);
        if (rc) {
            t->ops.resize(before);      // all or nothing
            t->n_channels = ch_before;
            return fail(rc, "op " + std::to_string(i) + ": " + vqd_last_error());
        }
    }
    return VQD_OK;
}

int vqd_traj_add_unitary(vqd_traj *t, int k, const int *targets, const double *u)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    if (k < 1 || k > 4) return fail(VQD_E_SIZE, "unitary needs k in [1, 4]");
    if (int rc = check_targets(t->n, k, targets)) return rc;
    if (!u) return fail(VQD_E_ARG, "null matrix");
    const size_t cnt = size_t(1) << (2 * k);
    if (!all_finite(u, 2 * cnt)) return fail(VQD_E_ARG, "non-finite matrix entry");
    TIn op;
    if (int rc = make_gate(k, targets, read_complex(u, cnt), op)) return rc;
    return traj_push(t, std::move(op));
}

int vqd_traj_add_kraus(vqd_traj *t, int k, const int *targets, int nk, const double *kraus)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    if (k < 1 || k > 2) return fail(VQD_E_SIZE, "Kraus maps need k in [1, 2]");
    if (nk < 1 || nk > kTrajMaxKraus) return fail(VQD_E_SIZE, "need 1 to 16 Kraus operators");
    if (int rc = check_targets(t->n, k, targets)) return rc;
    if (!kraus) return fail(VQD_E_ARG, "null Kraus operators");
    const size_t cnt = size_t(1) << (2 * k);
    if (!all_finite(kraus, 2 * cnt * nk)) return fail(VQD_E_ARG, "non-finite Kraus entry");
    TIn op;
    op.k = k;
    for (int j = 0; j < k; ++j) op.q[j] = targets[j];
    op.chan = true;
    for (int i = 0; i < nk; ++i) op.K.push_back(read_complex(kraus + 2 * cnt * i, cnt));
    return traj_push(t, std::move(op));
}

int vqd_traj_plan(vqd_traj *t)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    return plan(t);
}

int vqd_traj_export(const vqd_traj *t, void *buf, size_t cap, size_t *needed)
{
    clear_error();
    if (!t || !needed) return fail(VQD_E_ARG, "null argument");
    if (t->phases.empty()) return fail(VQD_E_STATE, "trajectory program not planned");
    const uint32_t head[10] = {0x54445156u, 1u, (uint32_t)t->n, (uint32_t)t->n_eff, (uint32_t)t->n_channels,
                               (uint32_t)t->phases.size(), (uint32_t)t->kops.size(), (uint32_t)t->pool.size(),
                               (uint32_t)sizeof(TPhase), (uint32_t)sizeof(TOp)};
    const size_t b_ph = t->phases.size() * sizeof(TPhase), b_op = t->kops.size() * sizeof(TOp);
    const size_t total = sizeof(head) + b_ph + b_op + t->pool.size() * 16;
    *needed = total;
    if (!buf) return VQD_OK;
    if (cap < total) return fail(VQD_E_SIZE, "export buffer too small");
    char *o = static_cast<char *>(buf);
    std::memcpy(o, head, sizeof(head));
    o += sizeof(head);
    std::memcpy(o, t->phases.data(), b_ph);
    o += b_ph;
    if (b_op) std::memcpy(o, t->kops.data(), b_op);
    o += b_op;
    for (const cd &z : t->pool) {
        const double v[2] = {z.real(), z.imag()};
        std::memcpy(o, v, sizeof(v));
        o += sizeof(v);
    }
    return VQD_OK;
}

int vqd_traj_compile(vqd_traj *t)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    if (int rc = plan(t)) return rc;
    if (int rc = upload(t)) return rc;
    (void)hipGetDevice(&t->device);
    t->compiled = true;
    return VQD_OK;
}

int vqd_traj_info_get(const vqd_traj *t, vqd_traj_info *out)
{
    clear_error();
    if (!t || !out) return fail(VQD_E_ARG, "null argument");
    out->n = t->n;
    out->n_ops = (int)t->ops.size();
    out->n_channels = t->n_channels;
    out->n_phases = (int)t->phases.size();
    out->n_kernel_ops = (int)t->kops.size();
    out->n_mixed = t->n_mixed;
    out->n_general = t->n_general;
    out->fma_per_amp = t->fma_per_amp;
    return VQD_OK;
}

int vqd_traj_run(vqd_traj *t, const double *uniforms, long long count, double *z_out, double *norm_out,
                 double *state_out, void *hip_stream)
{
    clear_error();
    if (!t) return fail(VQD_E_ARG, "null trajectory program");
    if (!t->compiled) return fail(VQD_E_STATE, "trajectory program not compiled");
    if (count < 0) return fail(VQD_E_ARG, "negative trajectory count");
    if (count == 0) return VQD_OK;
    if (!z_out) return fail(VQD_E_ARG, "null z_out");
    if (t->n_channels > 0 && !uniforms) return fail(VQD_E_ARG, "null uniforms");
    int dev = -1;
    VQD_HIP(hipGetDevice(&dev));
    if (dev != t->device) return fail(VQD_E_ARG, "trajectory program compiled for another device");
    return launch_traj(t->d_phases, (uint32_t)t->phases.size(), t->d_ops, t->d_pool, t->n, t->n_eff,
                       (uint32_t)t->n_channels, uniforms, (uint64_t)count, z_out, norm_out, state_out,
                       (hipStream_t)hip_stream);
}

int vqd_traj_stats(const double *x, long long count, int m, double *mean, double *sem, void *hip_stream)
{
    clear_error();
    if (count < 1) return fail(VQD_E_ARG, "need at least one sample");
    if (m < 1) return fail(VQD_E_ARG, "need at least one column");
    if (!x || !mean || !sem) return fail(VQD_E_ARG, "null pointer");
    return launch_traj_stats(x, (uint64_t)count, m, mean, sem, (hipStream_t)hip_stream);
}

}  // extern "C"
