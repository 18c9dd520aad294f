// Gate matrices and channel superoperators built on the host in FP64.
//
// Gates follow the conventions R_sigma(theta) = exp(-i theta sigma / 2)
// (Rx is eq. u of Sec. 6 at zero detuning), the Rydberg/ZZ/exchange forms of
// Secs. 3.4 and 6, and the Kraus maps of Sec. 3 (eqs. depol1, depol2, deph1,
// deph2, damp, gdamp, bf, bf2, ampt1, depht2, depht2s, depolt1; gdamp with
// gamma(dt) = 1 - exp(-dt/T1)).  A two-qubit operator A on
// targets[0] and B on targets[1] has matrix kron(B, A) (targets[0] is the
// least significant bit of the index).
#include <array>
#include <cmath>
#include <cstring>

#include "vqd_internal.h"

namespace vqd {

namespace {

const cd I(0.0, 1.0);

using M2 = std::array<cd, 4>;

M2 pauli(int a)
{
    switch (a) {
    case 0: return {cd(1), cd(0), cd(0), cd(1)};
    case 1: return {cd(0), cd(1), cd(1), cd(0)};
    case 2: return {cd(0), -I, I, cd(0)};
    default: return {cd(1), cd(0), cd(0), cd(-1)};
    }
}

// kron(B, A): A on the low qubit, B on the high qubit.
std::vector<cd> kron2(const M2 &A, const M2 &B)
{
    std::vector<cd> M(16);
    for (int r1 = 0; r1 < 2; ++r1)
        for (int r0 = 0; r0 < 2; ++r0)
            for (int c1 = 0; c1 < 2; ++c1)
                for (int c0 = 0; c0 < 2; ++c0)
                    M[(r0 + 2 * r1) * 4 + (c0 + 2 * c1)] = A[r0 * 2 + c0] * B[r1 * 2 + c1];
    return M;
}

std::vector<cd> scaled(const std::vector<cd> &M, double s)
{
    std::vector<cd> o(M);
    for (auto &x : o) x *= s;
    return o;
}

std::vector<cd> m2v(const M2 &m) { return std::vector<cd>(m.begin(), m.end()); }

// Kraus sets of the named channels (each a list of d x d matrices).
int channel_kraus(int kind, const double *p, int &k, std::vector<std::vector<cd>> &Ks)
{
    Ks.clear();
    auto need_prob = [&](double x, double hi) {
        return std::isfinite(x) && x >= 0.0 && x <= hi;
    };
    switch (kind) {
    case VQD_K_DEPOL1: case VQD_K_DEPOL_T1: {
        double q = p[0];
        if (kind == VQD_K_DEPOL_T1) {
            if (!(p[1] > 0) || !(p[0] >= 0)) return fail(VQD_E_ARG, "depol_t1: need dt >= 0, T1 > 0");
            q = 0.75 * (1.0 - std::exp(-p[0] / p[1]));
        }
        if (!need_prob(q, 1.0)) return fail(VQD_E_ARG, "depol1: p outside [0, 1]");
        k = 1;
        Ks.push_back(scaled(m2v(pauli(0)), std::sqrt(1 - q)));
        for (int a = 1; a < 4; ++a) Ks.push_back(scaled(m2v(pauli(a)), std::sqrt(q / 3)));
        return VQD_OK;
    }
    case VQD_K_DEPOL2: {
        if (!need_prob(p[0], 1.0)) return fail(VQD_E_ARG, "depol2: p outside [0, 1]");
        k = 2;
        // operators in the order of the equation's terms (a trajectory's draw
        // depends on it): identity, sigma on the first target, sigma on the
        // second, then the products with the first target's Pauli outer
        Ks.push_back(scaled(kron2(pauli(0), pauli(0)), std::sqrt(1 - p[0])));
        for (int a = 1; a < 4; ++a) Ks.push_back(scaled(kron2(pauli(a), pauli(0)), std::sqrt(p[0] / 15)));
        for (int b = 1; b < 4; ++b) Ks.push_back(scaled(kron2(pauli(0), pauli(b)), std::sqrt(p[0] / 15)));
        for (int a = 1; a < 4; ++a)
            for (int b = 1; b < 4; ++b) Ks.push_back(scaled(kron2(pauli(a), pauli(b)), std::sqrt(p[0] / 15)));
        return VQD_OK;
    }
    case VQD_K_DEPH1: case VQD_K_DEPH_T2: case VQD_K_DEPH_T2S: {
        double q = p[0];
        if (kind == VQD_K_DEPH_T2) {
            if (!(p[1] > 0) || !(p[0] >= 0)) return fail(VQD_E_ARG, "deph_t2: need dt >= 0, T2 > 0");
            q = 0.5 * (1.0 - std::exp(-p[0] / p[1]));
        } else if (kind == VQD_K_DEPH_T2S) {
            if (!(p[1] > 0) || !(p[0] >= 0)) return fail(VQD_E_ARG, "deph_t2s: need dt >= 0, T2* > 0");
            const double r = p[0] / p[1];
            q = 0.5 * (1.0 - std::exp(-r * r));
        }
        if (!need_prob(q, 1.0)) return fail(VQD_E_ARG, "deph1: p outside [0, 1]");
        k = 1;
        Ks.push_back(scaled(m2v(pauli(0)), std::sqrt(1 - q)));
        Ks.push_back(scaled(m2v(pauli(3)), std::sqrt(q)));
        return VQD_OK;
    }
    case VQD_K_DEPH2: {
        if (!need_prob(p[0], 1.0)) return fail(VQD_E_ARG, "deph2: p outside [0, 1]");
        k = 2;
        Ks.push_back(scaled(kron2(pauli(0), pauli(0)), std::sqrt(1 - p[0])));
        Ks.push_back(scaled(kron2(pauli(3), pauli(0)), std::sqrt(p[0] / 3)));
        Ks.push_back(scaled(kron2(pauli(0), pauli(3)), std::sqrt(p[0] / 3)));
        Ks.push_back(scaled(kron2(pauli(3), pauli(3)), std::sqrt(p[0] / 3)));
        return VQD_OK;
    }
    case VQD_K_AMP: case VQD_K_AMP_T1: {
        double g = p[0];
        if (kind == VQD_K_AMP_T1) {
            if (!(p[1] > 0) || !(p[0] >= 0)) return fail(VQD_E_ARG, "amp_t1: need dt >= 0, T1 > 0");
            g = 1.0 - std::exp(-p[0] / p[1]);
        }
        if (!need_prob(g, 1.0)) return fail(VQD_E_ARG, "amp: p outside [0, 1]");
        k = 1;
        Ks.push_back({cd(1), cd(0), cd(0), cd(std::sqrt(1 - g))});
        Ks.push_back({cd(0), cd(std::sqrt(g)), cd(0), cd(0)});
        return VQD_OK;
    }
    case VQD_K_GAMP: case VQD_K_GAMP_T1: {
        double pp = p[0], g = p[1];
        if (kind == VQD_K_GAMP_T1) {
            if (!(p[2] > 0) || !(p[1] >= 0)) return fail(VQD_E_ARG, "gamp_t1: need dt >= 0, T1 > 0");
            g = 1.0 - std::exp(-p[1] / p[2]);
        }
        if (!need_prob(pp, 1.0) || !need_prob(g, 1.0)) return fail(VQD_E_ARG, "gamp: p, gamma outside [0, 1]");
        k = 1;
        double a = std::sqrt(pp), b = std::sqrt(1 - pp);
        Ks.push_back({cd(a), cd(0), cd(0), cd(a * std::sqrt(1 - g))});
        Ks.push_back({cd(0), cd(a * std::sqrt(g)), cd(0), cd(0)});
        Ks.push_back({cd(b * std::sqrt(1 - g)), cd(0), cd(0), cd(b)});
        Ks.push_back({cd(0), cd(0), cd(b * std::sqrt(g)), cd(0)});
        return VQD_OK;
    }
    case VQD_K_BITFLIP1: {
        if (!need_prob(p[0], 1.0)) return fail(VQD_E_ARG, "bitflip1: b outside [0, 1]");
        k = 1;
        Ks.push_back(scaled(m2v(pauli(0)), std::sqrt(1 - p[0])));
        Ks.push_back(scaled(m2v(pauli(1)), std::sqrt(p[0])));
        return VQD_OK;
    }
    case VQD_K_PARITY_DECAY: {
        // index a + 2 b of the ket |a b>; row-major 4x4 operators
        k = 2;
        for (int e : {0, 15, 5, 6}) {        // |00><00|, |11><11|, |10><10|, |10><01|
            std::vector<cd> K(16, cd(0));
            K[e] = 1;
            Ks.push_back(K);
        }
        return VQD_OK;
    }
    case VQD_K_BITFLIP2: {
        if (!need_prob(p[0], 1.0)) return fail(VQD_E_ARG, "bitflip2: b outside [0, 1]");
        k = 2;
        Ks.push_back(scaled(kron2(pauli(0), pauli(0)), std::sqrt(1 - p[0])));
        Ks.push_back(scaled(kron2(pauli(1), pauli(0)), std::sqrt(p[0] / 3)));
        Ks.push_back(scaled(kron2(pauli(0), pauli(1)), std::sqrt(p[0] / 3)));
        Ks.push_back(scaled(kron2(pauli(1), pauli(1)), std::sqrt(p[0] / 3)));
        return VQD_OK;
    }
    default:
        return fail(VQD_E_ARG, "not a channel kind: " + std::to_string(kind));
    }
}

// Driven two-level system (eq. u): with W = sqrt(Omega^2 + Delta^2) and
// a = W t / 2 the matrix is
//   [cos a - i Delta/W sin a,         -i Omega/W sin a e^{+i phi}]
//   [-i Omega/W sin a e^{-i phi},     cos a + i Delta/W sin a    ].
// frame = true multiplies row 0 by e^{+i a} and row 1 by e^{-i a}: the
// bystander seen from the driven qubit's frame (eq. off_resonant, phi = 0).
// W = 0 (no drive, no detuning) is the identity.
int rabi(double omega, double phi, double delta, double t, bool frame, std::vector<cd> &U)
{
    const double w = std::hypot(omega, delta);
    const double a = 0.5 * w * t;
    const double c = std::cos(a), s = std::sin(a);
    const double sw = (w > 0.0) ? s / w : 0.5 * t;     // sin(a)/W, its limit at W = 0
    const cd off = -I * (omega * sw);
    U = {cd(c, -delta * sw), off * std::exp(I * phi), off * std::exp(-I * phi), cd(c, delta * sw)};
    if (frame) {
        const cd e0 = std::exp(I * a), e1 = std::conj(e0);
        U[0] *= e0;      // row 0 (row-major)
        U[1] *= e0;
        U[2] *= e1;      // row 1
        U[3] *= e1;
    }
    return VQD_OK;
}

bool is_channel(int kind)
{
    return (kind >= VQD_K_DEPOL1 && kind <= VQD_K_GAMP_T1) || kind == VQD_K_PARITY_DECAY;
}

}  // namespace

void canonical_params(int kind, double *p)
{
    p[0] = p[1] = p[2] = p[3] = 0.0;
    switch (kind) {
    case VQD_K_SU2: p[0] = 0.31; p[1] = 0.52; p[2] = -0.73; p[3] = 0.44; break;
    case VQD_K_GAMP: p[0] = 0.83; p[1] = 0.11; break;
    case VQD_K_GAMP_T1: p[0] = 0.83; p[1] = 0.3; p[2] = 17.0; break;
    case VQD_K_AMP_T1: case VQD_K_DEPH_T2: case VQD_K_DEPH_T2S: case VQD_K_DEPOL_T1:
        p[0] = 0.3; p[1] = 17.0; break;
    case VQD_K_RABI: p[0] = 5.0; p[1] = 0.4; p[2] = 1.3; p[3] = 0.21; break;
    case VQD_K_OFFRES: p[0] = 5.0; p[1] = 2.7; p[2] = 0.21; break;
    case VQD_K_RX: case VQD_K_RY: case VQD_K_RZ: case VQD_K_CPHASE: case VQD_K_XX: case VQD_K_ZZ:
    case VQD_K_CRZ:
        p[0] = 0.7371; break;
    default: p[0] = 0.0123; break;        // channel probabilities
    }
}

int kind_arity(int kind, int *nq, int *np)
{
    static const int Q[VQD_K_COUNT] = {0, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2,
                                       1, 2, 1, 2, 1, 1, 1, 2, 1, 1, 1, 1, 1, 1, 1, 2, 2};
    static const int P[VQD_K_COUNT] = {0, 1, 1, 1, 0, 0, 0, 0, 4, 0, 1, 1, 1,
                                       1, 1, 1, 1, 1, 2, 1, 1, 2, 2, 2, 2, 3, 4, 3, 1, 0};
    if (kind <= 0 || kind >= VQD_K_COUNT) return -1;
    if (nq) *nq = Q[kind];
    if (np) *np = P[kind];
    return 0;
}

int kind_matrix(int kind, const double *p, std::vector<cd> &U, int &k)
{
    int nq = 0, np = 0;
    if (kind_arity(kind, &nq, &np) != 0 || is_channel(kind))
        return fail(VQD_E_ARG, "not a gate kind: " + std::to_string(kind));
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(p[i])) return fail(VQD_E_ARG, "non-finite gate parameter");
    k = nq;
    U.assign(size_t(1) << (2 * k), cd(0));
    switch (kind) {
    case VQD_K_RX: {
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        U = {cd(c), -I * s, -I * s, cd(c)};
        break;
    }
    case VQD_K_RY: {
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        U = {cd(c), cd(-s), cd(s), cd(c)};
        break;
    }
    case VQD_K_RZ:
        U = {std::exp(-I * (p[0] / 2)), cd(0), cd(0), std::exp(I * (p[0] / 2))};
        break;
    case VQD_K_H: {
        double r = 1.0 / std::sqrt(2.0);
        U = {cd(r), cd(r), cd(r), cd(-r)};
        break;
    }
    case VQD_K_X: U = m2v(pauli(1)); break;
    case VQD_K_Y: U = m2v(pauli(2)); break;
    case VQD_K_Z: U = m2v(pauli(3)); break;
    case VQD_K_SU2: {
        double nrm = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        if (!(nrm > 0)) return fail(VQD_E_ARG, "su2: zero quaternion");
        double a0 = p[0] / nrm, a1 = p[1] / nrm, a2 = p[2] / nrm, a3 = p[3] / nrm;
        // a0 I - i (a1 X + a2 Y + a3 Z)
        U = {cd(a0, -a3), cd(-a2, -a1), cd(a2, -a1), cd(a0, a3)};
        break;
    }
    case VQD_K_CZ:
        U[0] = 1; U[5] = 1; U[10] = 1; U[15] = -1;
        break;
    case VQD_K_CPHASE:
        U[0] = 1; U[5] = 1; U[10] = 1; U[15] = std::exp(I * p[0]);
        break;
    case VQD_K_XX: {
        // cos(theta/2) I - i sin(theta/2) X(x)X; X(x)X flips both index bits
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        for (int i = 0; i < 4; ++i) {
            U[i * 4 + i] = c;
            U[i * 4 + (i ^ 3)] = -I * s;
        }
        break;
    }
    case VQD_K_ZZ: {
        // exp(-i alpha Z(x)Z): phase e^{-i alpha} on even parity, e^{+i alpha} on odd
        for (int i = 0; i < 4; ++i) {
            int par = (i ^ (i >> 1)) & 1;
            U[i * 4 + i] = std::exp(-I * (par ? -p[0] : p[0]));
        }
        break;
    }
    case VQD_K_CRZ:
        // index b(control) + 2 b(target): the target's Rz acts where the control is 1
        U[0] = 1; U[5] = std::exp(-I * (p[0] / 2)); U[10] = 1; U[15] = std::exp(I * (p[0] / 2));
        break;
    case VQD_K_RABI:
        return rabi(p[0], p[1], p[2], p[3], false, U);
    case VQD_K_OFFRES:
        return rabi(p[0], 0.0, p[1], p[2], true, U);
    default:
        return fail(VQD_E_ARG, "not a gate kind");
    }
    return VQD_OK;
}

int kind_kraus(int kind, const double *p, std::vector<std::vector<cd>> &Ks, int &k)
{
    int nq = 0, np = 0;
    if (kind_arity(kind, &nq, &np) != 0 || !is_channel(kind))
        return fail(VQD_E_ARG, "not a channel kind: " + std::to_string(kind));
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(p[i])) return fail(VQD_E_ARG, "non-finite channel parameter");
    return channel_kraus(kind, p, k, Ks);
}

bool kind_is_channel(int kind) { return is_channel(kind); }

void unitary_to_superop(int k, const cd *U, std::vector<cd> &S)
{
    kraus_to_superop(k, 1, U, S);
}

void kraus_to_superop(int k, int nk, const cd *K, std::vector<cd> &S)
{
    const int d = 1 << k, D = d * d;
    S.assign(size_t(D) * D, cd(0));
    for (int j = 0; j < nk; ++j) {
        const cd *Kj = K + size_t(j) * d * d;
        for (int c2 = 0; c2 < d; ++c2)
            for (int r2 = 0; r2 < d; ++r2)
                for (int c = 0; c < d; ++c)
                    for (int r = 0; r < d; ++r)
                        S[size_t(r2 + d * c2) * D + (r + d * c)] +=
                            Kj[r2 * d + r] * std::conj(Kj[c2 * d + c]);
    }
}

int kind_superop(int kind, const double *p, std::vector<cd> &S, int &k)
{
    int nq = 0, np = 0;
    if (kind_arity(kind, &nq, &np) != 0) return fail(VQD_E_ARG, "unknown kind " + std::to_string(kind));
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(p[i])) return fail(VQD_E_ARG, "non-finite op parameter");
    if (!is_channel(kind)) {
        std::vector<cd> U;
        int rc = kind_matrix(kind, p, U, k);
        if (rc) return rc;
        unitary_to_superop(k, U.data(), S);
        return VQD_OK;
    }
    std::vector<std::vector<cd>> Ks;
    int rc = channel_kraus(kind, p, k, Ks);
    if (rc) return rc;
    const int d = 1 << k;
    std::vector<cd> flat;
    for (auto &m : Ks) flat.insert(flat.end(), m.begin(), m.end());
    kraus_to_superop(k, int(Ks.size()), flat.data(), S);
    (void)d;
    return VQD_OK;
}

void fill_superop_op(LOp &op, int k, const int *targets, const cd *S)
{
    op.k = k;
    for (int j = 0; j < 4; ++j) op.q[j] = (j < k) ? targets[j] : 0;
    op.wide_unitary = false;
    op.U.clear();
    const int D = 1 << (2 * k);
    bool diag = true;
    for (int i = 0; i < D && diag; ++i)
        for (int j = 0; j < D; ++j)
            if (i != j && S[size_t(i) * D + j] != cd(0)) { diag = false; break; }
    op.diag = diag;
    if (diag) {
        op.D.resize(D);
        for (int i = 0; i < D; ++i) op.D[i] = S[size_t(i) * D + i];
        op.S.clear();
    } else {
        op.S.assign(S, S + size_t(D) * D);
        op.D.clear();
    }
}

LOp make_superop_op(int k, const int *targets, const cd *S)
{
    LOp op;
    fill_superop_op(op, k, targets, S);
    return op;
}

LOp make_unitary_op(int k, const int *targets, const cd *U)
{
    if (k <= 2) {
        std::vector<cd> S;
        unitary_to_superop(k, U, S);
        return make_superop_op(k, targets, S.data());
    }
    LOp op;
    op.k = k;
    for (int j = 0; j < k; ++j) op.q[j] = targets[j];
    op.wide_unitary = true;
    op.U.assign(U, U + (size_t(1) << (2 * k)));
    return op;
}

}  // namespace vqd

// ------------------------------------------------------- error parameters --
// App. B: average and entanglement fidelity, eq. (fidelities_relation); the
// depolarising + dephasing entanglement fidelity 1 - p - q + c p q, c = 4/3
// for one qubit (eq. fe1) and 16/15 for two; the split of a reported average
// fidelity into depolarising x eps and dephasing (1 - x) eps.
extern "C" {

int vqd_entanglement_fidelity(int nq, double p_depol, double p_deph, double *fe)
{
    vqd::clear_error();
    if (nq != 1 && nq != 2) return vqd::fail(VQD_E_ARG, "only one- and two-qubit gates");
    if (!fe) return vqd::fail(VQD_E_ARG, "null output");
    if (!std::isfinite(p_depol) || !std::isfinite(p_deph)) return vqd::fail(VQD_E_ARG, "non-finite parameter");
    const double c = nq == 1 ? 4.0 / 3.0 : 16.0 / 15.0;
    *fe = 1.0 - p_depol - p_deph + c * p_depol * p_deph;
    return VQD_OK;
}

int vqd_fidelity_to_errors(int nq, double fbar, double x, double *p_depol, double *p_deph)
{
    vqd::clear_error();
    if (nq != 1 && nq != 2) return vqd::fail(VQD_E_ARG, "only one- and two-qubit gates");
    if (!p_depol || !p_deph) return vqd::fail(VQD_E_ARG, "null output");
    if (!(x >= 0.0 && x <= 1.0)) return vqd::fail(VQD_E_ARG, "x outside [0, 1]");
    if (!(fbar <= 1.0) || !std::isfinite(fbar)) return vqd::fail(VQD_E_ARG, "fidelity above 1");
    const double d = nq == 1 ? 2.0 : 4.0;
    const double c = nq == 1 ? 4.0 / 3.0 : 16.0 / 15.0;
    const double fe = ((d + 1.0) * fbar - 1.0) / d;
    // 1 - eps + a eps^2 = fe with a = c x (1 - x): the smaller root, written
    // without cancellation
    const double a = c * x * (1.0 - x), delta = 1.0 - fe;
    const double disc = 1.0 - 4.0 * a * delta;
    if (delta < 0.0 || disc < 0.0) return vqd::fail(VQD_E_ARG, "no error parameters reach this fidelity");
    const double eps = 2.0 * delta / (1.0 + std::sqrt(disc));
    if (eps > 1.0) return vqd::fail(VQD_E_ARG, "no error parameters in [0, 1] reach this fidelity");
    *p_depol = x * eps;
    *p_deph = (1.0 - x) * eps;
    return VQD_OK;
}

double vqd_angle_scaled_error(double eps, double theta)
{
    return eps * std::fabs(theta) / 3.14159265358979323846;
}

int vqd_zz_crosstalk_strength(double J, double delta_ct, double alpha_c, double alpha_t, double *beta)
{
    vqd::clear_error();
    if (!beta) return vqd::fail(VQD_E_ARG, "null output");
    if (!std::isfinite(J) || !std::isfinite(delta_ct) || !std::isfinite(alpha_c) || !std::isfinite(alpha_t))
        return vqd::fail(VQD_E_ARG, "non-finite parameter");
    const double a = delta_ct - alpha_t, b = delta_ct + alpha_c;
    if (a == 0.0 || b == 0.0) return vqd::fail(VQD_E_ARG, "zero denominator");
    *beta = J * J * (1.0 / a - 1.0 / b);
    return VQD_OK;
}

}  // extern "C"
