"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here runs on a GPU.  Every oracle function is tied to at least one of:
a brute-force tensor contraction (n <= 4), a closed form, a value the paper
prints, an end point of a channel's parameter range, or a gate identity.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import channels as ch
from oracle.core import OracleDM
from oracle.emulator import emulate
from workloads import c1_line_circuit, random_matrix_ops
from tests import _brute as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_state(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    rho = A @ A.conj().T
    return rho / np.trace(rho)


def random_nonhermitian(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))


def oracle_with(rho):
    n = int(round(math.log2(rho.shape[0])))
    dm = OracleDM(n)
    dm.set(rho)
    return dm


# ------------------------------------------------------------ brute force --

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_matrix_and_kraus_match_bruteforce(n):
    """Random (non-unitary, non-TP) matrices and Kraus sets on random targets,
    applied to a non-Hermitian start so that a swapped or missing conjugate
    shows up."""
    rho = random_nonhermitian(n, 11 + n)
    dm = oracle_with(rho)
    ref = rho.copy()
    for kind, tg, params in random_matrix_ops(n, 24, seed=100 + n, max_k=min(2, n)):
        if kind == "matrix":
            dm.apply_matrix(tg, params[0])
            ref = bf.apply_op(ref, n, tg, params[0])
        else:
            dm.apply_kraus(tg, params)
            ref = bf.apply_kraus(ref, n, tg, params)
    scale = np.abs(ref).max()
    assert np.abs(dm.R - ref).max() <= 1e-12 * max(scale, 1.0)


@pytest.mark.parametrize("k", [3, 4])
def test_wide_ops_match_bruteforce(k):
    n = 4
    rng = np.random.default_rng(k)
    rho = random_nonhermitian(n, 3)
    tg = tuple(int(x) for x in rng.permutation(n)[:k])
    M = (rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))) / 4
    Ks = [(rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))) / 6
          for _ in range(2)]
    dm = oracle_with(rho)
    dm.apply_matrix(tg, M)
    dm.apply_kraus(tg, Ks)
    ref = bf.apply_kraus(bf.apply_op(rho, n, tg, M), n, tg, Ks)
    assert np.abs(dm.R - ref).max() <= 1e-12 * np.abs(ref).max()


def test_embedding_bit_order():
    """targets[0] is the least significant bit: X on qubit 2 of |0000> gives
    basis state 4; a 2-qubit matrix mapping index 1 -> 2 on targets (3, 0)
    moves a 1 from qubit 3 to qubit 0."""
    dm = OracleDM(4)
    dm.apply_matrix((2,), ch.X)
    assert dm.R[4, 4] == 1.0
    M = np.zeros((4, 4), dtype=complex)
    M[2, 1] = 1.0   # |b0=1,b1=0> -> |b0=0,b1=1>, b0 on target 3, b1 on target 0
    for i in (0, 1, 3):
        M[i, i] = 1.0
    M[1, 2] = 1.0
    dm.init_basis(8)
    dm.apply_matrix((3, 0), M)
    assert dm.R[1, 1] == 1.0


@pytest.mark.parametrize("n", [2, 3, 4])
def test_readouts_match_bruteforce(n):
    rho = random_state(n, 7 * n)
    dm = oracle_with(rho)
    D = 1 << n
    assert abs(dm.trace() - np.trace(rho)) < 1e-14
    assert np.allclose(dm.probs(), np.real(np.diag(rho)), atol=1e-15)
    Zs = [np.real(np.trace(bf.pauli_string([3 if q == i else 0 for q in range(n)]) @ rho))
          for i in range(n)]
    assert np.allclose(dm.expec_z(), Zs, atol=1e-14)
    pairs = [(i, j) for i in range(n) for j in range(n) if i != j]
    ZZ = [np.real(np.trace(bf.pauli_string([3 if q in (i, j) else 0 for q in range(n)]) @ rho))
          for i, j in pairs]
    assert np.allclose(dm.expec_zz(pairs), ZZ, atol=1e-14)
    assert abs(dm.purity() - np.real(np.trace(rho @ rho))) < 1e-14
    rng = np.random.default_rng(n)
    for _ in range(12):
        codes = rng.integers(0, 4, n)
        ref = np.trace(bf.pauli_string(codes) @ rho)
        assert abs(dm.expec_pauli(codes) - ref) < 1e-14
    assert D == rho.shape[0]


def test_initial_states():
    dm = OracleDM(3)
    dm.init_basis(5)
    assert dm.R[5, 5] == 1 and np.count_nonzero(dm.R) == 1
    p0 = np.array([0.9, 0.8, 0.7])
    dm.init_product_diag(p0)
    # eq. (thermalstate): tensor product of p|0><0| + (1-p)|1><1|
    ref = np.array([[1.0]])
    for p in p0:
        ref = np.kron(np.diag([p, 1 - p]), ref)
    assert np.allclose(dm.R, ref, atol=1e-16)


# --------------------------------------------------- pure-state reference --

def test_noise_free_circuit_matches_state_vector():
    """Gates only: rho must equal |psi><psi| of an independent state-vector run."""
    n = 5
    ops = [op for op in c1_line_circuit(n=n, n_gates=60) if op[0] in ("rx", "ry", "rz", "cz")]
    dm = emulate(n, ops)
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    for kind, tg, params in ops:
        U = ch.gate_matrix(kind, params)
        psi = bf.embed(n, tg, U) @ psi
    assert np.abs(dm.R - np.outer(psi, psi.conj())).max() < 1e-13
    assert abs(dm.purity() - 1) < 1e-13


# ------------------------------------------------------ textbook states --

def bell_ops(a, b):
    """H on a, then CNOT(a -> b) written as H_b CZ H_b."""
    return [("h", (a,), ()), ("h", (b,), ()), ("cz", (a, b), ()), ("h", (b,), ())]


@pytest.mark.parametrize("n", [2, 3, 5])
def test_ghz(n):
    ops = [("h", (0,), ())]
    for q in range(1, n):
        ops += [("h", (q,), ()), ("cz", (q - 1, q), ()), ("h", (q,), ())]
    dm = emulate(n, ops)
    D = 1 << n
    nz = np.argwhere(np.abs(dm.R) > 1e-12)
    assert sorted(map(tuple, nz)) == [(0, 0), (0, D - 1), (D - 1, 0), (D - 1, D - 1)]
    assert np.allclose(dm.R[[0, 0, D - 1, D - 1], [0, D - 1, 0, D - 1]], 0.5, atol=1e-14)
    assert np.allclose(dm.expec_z(), 0, atol=1e-14)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    assert np.allclose(dm.expec_zz(pairs), 1, atol=1e-14)
    assert abs(dm.purity() - 1) < 1e-14


# -------------------------------------------------------- closed forms --

@pytest.mark.parametrize("p,k", [(0.01, 7), (0.2, 3), (0.75, 2)])
def test_depol1_purity_decay(p, k):
    """Each depol1(p) scales the Bloch vector by 1 - 4p/3, so k applications on
    |0> give purity (1 + (1-4p/3)^(2k)) / 2 (on one qubit of a 3-qubit product)."""
    dm = emulate(3, [("depol1", (1,), (p,))] * k)
    assert abs(dm.purity() - (1 + (1 - 4 * p / 3) ** (2 * k)) / 2) < 1e-14


@pytest.mark.parametrize("p,k", [(0.05, 4), (0.3, 2)])
def test_dephasing_x_decay(p, k):
    """deph1(p) k times on |+>: <X> = (1-2p)^k."""
    dm = emulate(2, [("h", (0,), ())] + [("deph1", (0,), (p,))] * k)
    assert abs(dm.expec_pauli([1, 0]).real - (1 - 2 * p) ** k) < 1e-14


def test_t1_t2_exponentials():
    """eq. (ampt1) compounded over total time t: P(1) = exp(-t/T1) exactly.
    With eq. (depht2) as well, on |+>: <X> = exp(-t/T2) exp(-t/(2 T1))."""
    T1, T2, dt, steps = 100.0, 50.0, 0.5, 40
    t = dt * steps
    dm = emulate(2, [("x", (1,), ())] + [("amp_t1", (1,), (dt, T1))] * steps)
    assert abs(dm.probs()[2] - math.exp(-t / T1)) < 1e-14
    ops = [("h", (0,), ())]
    for _ in range(steps):
        ops += [("amp_t1", (0,), (dt, T1)), ("deph_t2", (0,), (dt, T2))]
    dm = emulate(2, ops)
    assert abs(dm.expec_pauli([1, 0]).real - math.exp(-t / T2) * math.exp(-t / (2 * T1))) < 1e-14


@pytest.mark.parametrize("p", [0.0, 0.05, 0.5, 15 / 16])
def test_depol2_on_bell(p):
    """depol2(p) on |Phi+>: fidelity 1 - 4p/5 (3 of the 15 Paulis stabilise it)."""
    dm = emulate(2, bell_ops(0, 1) + [("depol2", (0, 1), (p,))])
    phi = np.array([1, 0, 0, 1]) / math.sqrt(2)
    assert abs(phi @ dm.R @ phi - (1 - 4 * p / 5)) < 1e-14


@pytest.mark.parametrize("p,q", [(0.07, 0.13), (0.0, 0.3), (0.25, 0.0), (0.5, 0.75)])
def test_entanglement_fidelity_1q(p, q):
    """App. B eq. (fe1): F_e of deph(p) o depol(q) on one half of |Phi+> is
    1 - p - q + 4/3 p q."""
    dm = emulate(2, bell_ops(0, 1) + [("depol1", (0,), (q,)), ("deph1", (0,), (p,))])
    phi = np.array([1, 0, 0, 1]) / math.sqrt(2)
    assert abs(phi @ dm.R @ phi - (1 - p - q + 4 / 3 * p * q)) < 1e-14


@pytest.mark.parametrize("p,q", [(0.07, 0.13), (0.3, 0.6)])
def test_entanglement_fidelity_2q(p, q):
    """App. B: on two Bell pairs (qubits 0-2 and 1-3), deph2(p) o depol2(q) on
    (0, 1) gives F_e = 1 - p - q + 16/15 p q."""
    ops = bell_ops(0, 2) + bell_ops(1, 3) + [("depol2", (0, 1), (q,)), ("deph2", (0, 1), (p,))]
    dm = emulate(4, ops)
    ref = emulate(4, bell_ops(0, 2) + bell_ops(1, 3))
    F = np.real(np.trace(ref.R @ dm.R))
    assert abs(F - (1 - p - q + 16 / 15 * p * q)) < 1e-14


def test_ion_bell_pair_psi_minus_population():
    """The paper prints 0.046 for the |Psi^-> population of the raw ion Bell pair."""
    g = json.load(open(os.path.join(GOLDEN, "ion_bell_psi_minus.json")))
    psi_p = np.array([0, 1, 1, 0]) / math.sqrt(2)
    psi_m = np.array([0, 1, -1, 0]) / math.sqrt(2)
    base = bell_ops(0, 1) + [("x", (1,), ())]          # |Psi+>

    def state(eps):
        return emulate(2, base + [("depol2", (0, 1), (g["depol_fraction"] * eps,)),
                                  ("deph2", (0, 1), (g["deph_fraction"] * eps,))]).R

    eps = brentq(lambda e: np.real(psi_p @ state(e) @ psi_p) - g["fid_ent"], 0.0, 0.5, xtol=1e-15)
    pm = np.real(psi_m @ state(eps) @ psi_m)
    assert abs(pm - g["psi_minus_population"]) <= g["abs_tolerance"]


# ------------------------------------------------------ channel end points --

def test_channel_end_points():
    rho = random_state(2, 5)
    # eq. (damp): p = 1 sends every state of that qubit to |0><0|
    dm = oracle_with(rho)
    dm.apply_kraus((0,), ch.amp(1.0))
    red = dm.R.reshape(2, 2, 2, 2).trace(axis1=0, axis2=2)   # trace out qubit 1
    assert np.allclose(red, np.diag([1, 0]), atol=1e-15)
    # eq. (depol1) at p = 3/4: the qubit becomes maximally mixed
    dm = oracle_with(rho)
    dm.apply_kraus((1,), ch.depol1(0.75))
    red0 = dm.R.reshape(2, 2, 2, 2).trace(axis1=1, axis2=3)  # trace out qubit 0
    assert np.allclose(red0, np.eye(2) / 2, atol=1e-15)
    # eq. (depol2) at p = 15/16: the pair becomes I/4
    dm = oracle_with(rho)
    dm.apply_kraus((0, 1), ch.depol2(15 / 16))
    assert np.allclose(dm.R, np.eye(4) / 4, atol=1e-15)
    # eq. (deph1) at p = 1/2: coherences of that qubit vanish
    dm = oracle_with(rho)
    dm.apply_kraus((0,), ch.deph1(0.5))
    R4 = dm.R.reshape(2, 2, 2, 2)        # (r1, r0, c1, c0)
    assert np.allclose(R4[:, 0, :, 1], 0, atol=1e-16) and np.allclose(R4[:, 1, :, 0], 0, atol=1e-16)
    # eq. (bf) at b = 1/2: <Z> of that qubit is 0
    dm = oracle_with(rho)
    dm.apply_kraus((1,), ch.bitflip1(0.5))
    assert abs(dm.expec_z()[1]) < 1e-15
    # eq. (gdamp) with gamma = 1 sends the qubit to p|0><0| + (1-p)|1><1|
    dm = oracle_with(rho)
    dm.apply_kraus((0,), ch.gamp(0.8, 1.0))
    red = dm.R.reshape(2, 2, 2, 2).trace(axis1=0, axis2=2)
    assert np.allclose(red, np.diag([0.8, 0.2]), atol=1e-15)


def test_cptp_sets_and_cptn_leakage():
    for Ks in (ch.depol1(0.1), ch.depol2(0.2), ch.deph1(0.3), ch.deph2(0.4), ch.amp(0.5),
               ch.gamp(0.7, 0.2), ch.bitflip1(0.1), ch.bitflip2(0.2)):
        d = Ks[0].shape[0]
        assert np.allclose(sum(K.conj().T @ K for K in Ks), np.eye(d), atol=1e-15)
    # eq. (czleak): K = diag(1, sqrt(1-a), sqrt(1-a), sqrt(1-b)) is trace
    # decreasing; the trace lost from |11> is exactly b
    a, b = 0.02, 0.05
    K = np.diag([1, math.sqrt(1 - a), math.sqrt(1 - a), math.sqrt(1 - b)])
    dm = OracleDM(2)
    dm.init_basis(3)
    dm.apply_kraus((0, 1), [K])
    assert abs(dm.trace() - (1 - b)) < 1e-15


def test_silicon_parity_decay_map():
    """Sec. 7: the parity read-out's decay map is trace preserving, sends
    |0_i 1_j> to |1_i 0_j> (ket |a b> on (i, j) means a on i), and leaves
    |00>, |11> and |10> unchanged, so it keeps each parity."""
    Ks = ch.parity_decay()
    assert np.abs(sum(K.conj().T @ K for K in Ks) - np.eye(4)).max() == 0
    for start, end in ((0b100, 0b010), (0b000, 0b000), (0b110, 0b110), (0b010, 0b010)):
        dm = OracleDM(3)
        dm.init_basis(start)         # bit 1 is qubit i, bit 2 qubit j
        dm.apply_kraus((1, 2), Ks)
        assert abs(dm.R[end, end] - 1) < 1e-15, (start, end)


# ------------------------------------------------------- gate identities --

def same_up_to_phase(A, B):
    k = np.argmax(np.abs(B))
    ph = A.flat[k] / B.flat[k]
    return abs(abs(ph) - 1) < 1e-12 and np.allclose(A, ph * B, atol=1e-12)


@pytest.mark.parametrize("theta", [0.3, 1.7, 4.0])
def test_rx_is_raman_u_at_zero_detuning(theta):
    """Sec. 6 after eq. (u): U(0, 0, theta / Omega) is Rx(theta), here the
    matrix exponential exp(-i theta X / 2)."""
    from scipy.linalg import expm
    omega = 2.3
    assert np.abs(ch.gate_matrix("rabi", (omega, 0.0, 0.0, theta / omega))
                  - expm(-0.5j * theta * ch.X)).max() < 1e-14


def test_hadamard_from_raman_u():
    """Sec. 6 after eq. (u): U(0, Omega, pi / W) is a Hadamard gate (up to a
    global phase)."""
    omega = 1.1
    w = math.sqrt(2) * omega
    assert same_up_to_phase(ch.gate_matrix("rabi", (omega, 0.0, omega, math.pi / w)), (ch.X + ch.Z) / math.sqrt(2))


@pytest.mark.parametrize("omega,phi,delta,t", [(2.3, 0.0, 0.0, 0.4), (1.7, 0.9, -0.6, 1.3),
                                               (0.4, -2.2, 3.1, 2.9), (5.0, 0.4, 1.3, 0.21)])
def test_raman_u_is_the_driven_two_level_propagator(omega, phi, delta, t):
    """eq. (u) is the propagator of the drive Hamiltonian
    (Omega cos(phi) X - Omega sin(phi) Y + Delta Z) / 2 for a time t, here by
    scipy's matrix exponential; a sign of phi or Delta, a transposed
    off-diagonal or a dropped factor 1/W each fail it."""
    from scipy.linalg import expm
    H = 0.5 * (omega * math.cos(phi) * ch.X - omega * math.sin(phi) * ch.Y + delta * ch.Z)
    assert np.abs(ch.gate_matrix("rabi", (omega, phi, delta, t)) - expm(-1j * t * H)).max() < 1e-13
    assert np.abs(ch.gate_matrix("rabi", (0.0, phi, 0.0, t)) - np.eye(2)).max() == 0.0


@pytest.mark.parametrize("omega,delta,t", [(1.0, 2.0, 0.7), (5.0, 2.7, 0.21), (0.3, 40.0, 1.9)])
def test_off_resonant_is_the_bystander_in_the_drive_frame(omega, delta, t):
    """eq. (off_resonant): the detuned propagator of the same Hamiltonian
    with phi = 0, followed by the frame rotation exp(i W t Z / 2) of the
    driven qubit (W = sqrt(Omega^2 + Delta^2)); unitary."""
    from scipy.linalg import expm
    w = math.sqrt(omega ** 2 + delta ** 2)
    H = 0.5 * (omega * ch.X + delta * ch.Z)
    ref = expm(0.5j * w * t * ch.Z) @ expm(-1j * t * H)
    U = ch.gate_matrix("offres", (omega, delta, t))
    assert np.abs(U - ref).max() < 1e-13
    assert np.abs(U.conj().T @ U - np.eye(2)).max() < 1e-14


def test_off_resonant_without_drive_is_identity():
    """An undriven bystander (Omega = 0, Delta > 0) receives no operation: the
    detuning phase and the frame rotation cancel."""
    for delta, t in ((0.5, 3.0), (7.0, 0.11)):
        assert np.abs(ch.gate_matrix("offres", (0.0, delta, t)) - np.eye(2)).max() < 1e-15


def test_rydberg_cz_phi_zero_is_cz():
    phi = 0.0
    czphi = np.diag([1, np.exp(1j * phi), np.exp(1j * phi), np.exp(1j * (2 * phi - math.pi))])
    assert np.allclose(czphi, ch.gate_matrix("cz", ()), atol=1e-15)


def test_exchange_at_pi_is_swap():
    """eq. (exchange_pauli) at theta = pi is SWAP up to a global phase."""
    G = sum(ch.on2(P, P) for P in (ch.X, ch.Y, ch.Z))
    from scipy.linalg import expm
    U = expm(-1j * G * math.pi / 4)
    dm = OracleDM(2)
    dm.init_basis(0b01)
    dm.apply_matrix((0, 1), U)
    assert abs(dm.R[0b10, 0b10] - 1) < 1e-14


def test_off_resonant_tends_to_identity():
    """Sec. 3.3: eq. (off_resonant) approaches the identity as the detuning
    grows, here within Omega / Delta, and a state's populations stay put."""
    omega, t = 1.0, 3.0
    dm = OracleDM(1)
    dm.apply_matrix((0,), ch.gate_matrix("h", ()))
    ref = dm.R.copy()
    for delta in (1e2, 1e4):
        U = ch.gate_matrix("offres", (omega, delta, t))
        assert np.abs(U - np.eye(2)).max() <= omega / delta
        d2 = OracleDM(1)
        d2.set(ref)
        d2.apply_matrix((0,), U)
        assert abs(d2.R[0, 0] - ref[0, 0]) < omega / delta


def test_xx_at_half_pi_is_maximally_entangling():
    dm = emulate(2, [("xx", (0, 1), (math.pi / 2,))])
    # (|00> - i|11>)/sqrt2: populations 1/2, 1/2 and |coherence| 1/2
    assert abs(dm.R[0, 0] - 0.5) < 1e-15 and abs(dm.R[3, 3] - 0.5) < 1e-15
    assert abs(abs(dm.R[0, 3]) - 0.5) < 1e-15


# ------------------------------------------------------------- invariants --

def test_invariants_on_noisy_circuit():
    """CPTP stream: trace 1, Hermitian, purity in (0, 1]."""
    dm = emulate(6, c1_line_circuit(n=6, n_gates=60))
    assert abs(dm.trace() - 1) < 1e-13
    assert np.abs(dm.R - dm.R.conj().T).max() < 1e-14
    assert 0 < dm.purity() <= 1 + 1e-14


def test_unital_channels_do_not_raise_purity():
    rho = random_state(3, 9)
    dm = oracle_with(rho)
    last = dm.purity()
    for Ks, tg in ((ch.depol1(0.1), (0,)), (ch.deph2(0.2), (1, 2)), (ch.bitflip2(0.3), (2, 0)),
                   (ch.depol2(0.05), (0, 2))):
        dm.apply_kraus(tg, Ks)
        cur = dm.purity()
        assert cur <= last + 1e-15
        last = cur


# ------------------------------------------- builders with their own pins --

@pytest.mark.parametrize("seed", range(6))
def test_su2_draw_is_special_unitary(seed):
    """The Haar SU(2) draw of the grid circuit's one-qubit layers: a
    normalised Gaussian quaternion gives a unitary of determinant 1, and
    scaling the four draws does not change the gate."""
    g = np.random.default_rng(seed).standard_normal(4)
    U = ch.su2_from_gaussians(g)
    assert np.abs(U.conj().T @ U - np.eye(2)).max() < 1e-15
    assert abs(np.linalg.det(U) - 1) < 1e-15
    assert np.abs(ch.su2_from_gaussians(3.7 * g) - U).max() < 1e-15


def test_su2_draw_unit_quaternions():
    """The four unit quaternions give I, -iX, -iY, -iZ, written out entry by
    entry."""
    i = 1j
    want = {
        (1, 0, 0, 0): [[1, 0], [0, 1]],
        (0, 1, 0, 0): [[0, -i], [-i, 0]],
        (0, 0, 1, 0): [[0, -1], [1, 0]],
        (0, 0, 0, 1): [[-i, 0], [0, i]],
    }
    for a, M in want.items():
        assert np.abs(ch.su2_from_gaussians(a) - np.array(M)).max() < 1e-15


@pytest.mark.parametrize("theta,axis", [(0.3, (1, 0, 0)), (2.1, (0, 1, 0)), (4.0, (0, 0, 1)),
                                        (1.234, (0.48, -0.6, 0.64))])
def test_su2_draw_is_a_rotation(theta, axis):
    """A quaternion (cos(theta/2), sin(theta/2) n) is the rotation
    exp(-i theta n.sigma / 2); the exponential is taken by scipy, so a wrong
    sign or a swapped Pauli in the quaternion form fails here."""
    from scipy.linalg import expm
    n = np.asarray(axis, dtype=float)
    n /= np.linalg.norm(n)
    a = np.concatenate([[math.cos(theta / 2)], math.sin(theta / 2) * n])
    G = n[0] * ch.X + n[1] * ch.Y + n[2] * ch.Z
    assert np.abs(ch.su2_from_gaussians(a) - expm(-0.5j * theta * G)).max() < 1e-14


def test_cphase_at_pi_is_cz():
    """Sec. 7 (silicon native operations): CZ is CPh(theta) at theta = pi."""
    assert np.abs(ch.gate_matrix("cphase", (math.pi,)) - np.diag([1, 1, 1, -1])).max() < 1e-15


@pytest.mark.parametrize("phi", [0.4, 1.9, -2.5])
def test_cphase_moves_only_the_one_one_phase(phi):
    """CPh(phi) on |++>: the state is (|00>+|01>+|10>+e^{i phi}|11>)/2, so
    rho_{00,11} = e^{-i phi}/4 and every coherence that does not involve
    |11> stays 1/4."""
    h = ch.gate_matrix("h", ())
    dm = emulate(2, [("h", (0,), ()), ("h", (1,), ()), ("cphase", (0, 1), (phi,))])
    R = dm.R
    assert abs(R[0, 3] - np.exp(-1j * phi) / 4) < 1e-15
    assert abs(R[3, 0] - np.exp(1j * phi) / 4) < 1e-15
    for r in range(3):
        for c in range(3):
            assert abs(R[r, c] - 0.25) < 1e-15
    assert np.abs(h @ h - np.eye(2)).max() < 1e-15


@pytest.mark.parametrize("b", [0.05, 0.3, 0.75])
def test_bitflip2_populations_from_zero(b):
    """eq. (bf2) on |00>: populations 1-b on 00 and b/3 on each of 10, 01,
    11.  X_i and X_iX_j both flip Z_i, so <Z_i> = <Z_j> = 1 - 4b/3, and
    <Z_i Z_j> = 1 - b - b/3 = 1 - 4b/3 as well."""
    dm = emulate(2, [("bitflip2", (0, 1), (b,))])
    p = dm.probs()
    assert np.abs(p - np.array([1 - b, b / 3, b / 3, b / 3])).max() < 1e-15
    assert abs(dm.expec_zz([(0, 1)])[0] - (1 - 4 * b / 3)) < 1e-15
    assert np.abs(dm.expec_z() - (1 - 4 * b / 3)).max() < 1e-15


@pytest.mark.parametrize("b", [0.1, 0.5])
def test_bitflip2_keeps_plus_plus(b):
    """eq. (bf2) holds only X errors, and |++> is an eigenstate of X_i, X_j
    and X_iX_j: the state is unchanged.  A Y or Z in place of an X would move
    it."""
    ops = [("h", (0,), ()), ("h", (1,), ())]
    ref = emulate(2, ops).R
    got = emulate(2, ops + [("bitflip2", (0, 1), (b,))]).R
    assert np.abs(got - ref).max() < 1e-15
    # a coherent state off the X axis does move: |+i> on qubit 0
    ops_y = [("h", (0,), ()), ("rz", (0,), (math.pi / 2,))]
    a = emulate(2, ops_y).R
    m = emulate(2, ops_y + [("bitflip2", (0, 1), (b,))]).R
    # X_i and X_iX_j (weight 2b/3) flip <Y_0>: it scales by 1 - 4b/3
    y0 = lambda R: 2 * R[1, 0].imag
    assert abs(y0(a) - 1) < 1e-15
    assert abs(y0(m) - (1 - 4 * b / 3)) < 1e-15


@pytest.mark.parametrize("theta", [0.2, 1.0, math.pi / 2, 2.8])
def test_xx_sign_of_the_exponent(theta):
    """XX(theta) = exp(-i theta/2 X(x)X) (reading of the Moelmer-Soerensen
    gate) takes |00> to cos(theta/2)|00> - i sin(theta/2)|11>, so
    rho_{00,11} = i sin(theta)/2: its imaginary part is positive on
    (0, pi).  The opposite sign of the exponent flips it."""
    R = emulate(2, [("xx", (0, 1), (theta,))]).R
    assert abs(R[0, 3] - 0.5j * math.sin(theta)) < 1e-15
    assert R[0, 3].imag > 0
    assert abs(R[0, 0] - math.cos(theta / 2) ** 2) < 1e-15
    assert abs(R[3, 3] - math.sin(theta / 2) ** 2) < 1e-15
