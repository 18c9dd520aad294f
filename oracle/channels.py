"""The oracle's own gate and channel builders -- TEST INFRASTRUCTURE.

Each builder returns either ``("matrix", M)`` (applied as M rho M^dagger) or
``("kraus", [K_0, K_1, ...])``.  Matrices act on the op's qubits with
``qubits[0]`` as the least significant bit of the matrix index, so a product
A_{q0} B_{q1} is ``np.kron(B, A)``.

Rotations are written as matrix exponentials of their generators (scipy's
``expm``), the channels as the Kraus sets of the paper's maps.  Citations are
to sections and equations of the paper.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = (I2, X, Y, Z)


def on2(a, b):
    """Operator ``a`` on qubits[0] and ``b`` on qubits[1] (qubits[0] = LSB)."""
    return np.kron(b, a)


# ---------------------------------------------------------------- gates --

def rot(P, theta):
    """exp(-i theta P / 2); Rx is eq. (u) of Sec. 6 at Delta = 0, t = theta/Omega."""
    return expm(-0.5j * theta * P)


def su2_from_gaussians(g):
    """Haar SU(2) element from a normalised 4-Gaussian quaternion a:
    U = a0 I - i (a1 X + a2 Y + a3 Z)."""
    a = np.asarray(g, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return a[0] * I2 - 1j * (a[1] * X + a[2] * Y + a[3] * Z)


def gate_matrix(kind, params):
    if kind == "rx":
        return rot(X, params[0])
    if kind == "ry":
        return rot(Y, params[0])
    if kind == "rz":
        return rot(Z, params[0])
    if kind == "h":
        return (X + Z) / math.sqrt(2.0)
    if kind == "x":
        return X.copy()
    if kind == "y":
        return Y.copy()
    if kind == "z":
        return Z.copy()
    if kind == "su2":
        return su2_from_gaussians(params)
    if kind == "cz":
        # |1><1| on both qubits picks up a sign
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if kind == "cphase":
        return np.diag([1, 1, 1, np.exp(1j * params[0])]).astype(np.complex128)
    if kind == "xx":
        # Moelmer-Soerensen XX(theta) = exp(-i theta/2 X(x)X)
        return expm(-0.5j * params[0] * on2(X, X))
    if kind == "zz":
        # ZZ crosstalk exp(-i alpha Z_p Z_q), eq. (weak_dephasing_zz) of Sec. 3.4
        return expm(-1j * params[0] * on2(Z, Z))
    if kind == "crz":
        # eq. (weak_dephasing): the target (qubits[1]) turns by Rz(alpha) where
        # the control (qubits[0], the low index bit) is 1
        a = params[0]
        return np.diag([1, np.exp(-0.5j * a), 1, np.exp(0.5j * a)]).astype(np.complex128)
    if kind == "rabi":
        return rabi_u(*params)
    if kind == "offres":
        return off_resonant(*params)
    if kind == "matrix":
        return np.asarray(params[0], dtype=np.complex128)
    raise KeyError(kind)


def rabi_u(omega, phi, delta, t):
    """eq. (u): U(phi, Delta, t) of a two-level system driven at Rabi
    frequency omega with phase phi and detuning Delta for a time t, with
    the generalised frequency W = sqrt(omega^2 + Delta^2).  Reading: at
    W = 0 (no drive, no detuning) the matrix is its limit, the identity."""
    W = math.sqrt(omega * omega + delta * delta)
    if W == 0.0:
        return I2.copy()
    c, s = math.cos(W * t / 2), math.sin(W * t / 2)
    return np.array([[c - 1j * delta / W * s, -1j * omega / W * s * np.exp(1j * phi)],
                     [-1j * omega / W * s * np.exp(-1j * phi), c + 1j * delta / W * s]])


def off_resonant(omega, delta, t):
    """eq. (off_resonant): the unitary a passive qubit detuned by delta from
    a qubit driven at Rabi frequency omega for a time t undergoes, written in
    the driven qubit's frame, with W = sqrt(omega^2 + delta^2).  Reading: at
    W = 0 the identity, its limit."""
    W = math.sqrt(omega * omega + delta * delta)
    if W == 0.0:
        return I2.copy()
    c, s = math.cos(W * t / 2), math.sin(W * t / 2)
    ep, em = np.exp(1j * W * t / 2), np.exp(-1j * W * t / 2)
    return np.array([[(c - 1j * delta / W * s) * ep, -1j * omega / W * s * ep],
                     [-1j * omega / W * s * em, (c + 1j * delta / W * s) * em]])


# ------------------------------------------------------------- channels --

def depol1(p):
    """eq. (depol1): (1-p) rho + p/3 sum_sigma sigma rho sigma."""
    return [math.sqrt(1 - p) * I2] + [math.sqrt(p / 3) * s for s in (X, Y, Z)]


def parity_decay():
    """Sec. 7 (eq. projmeas): the decay of |0_i 1_j> to |1_i 0_j> that comes
    with the silicon parity read-out, as the Kraus set {|00><00|, |11><11|,
    |10><10|, |10><01|}; ket |a b> has a on qubits[0], the low index bit."""
    def ket(a, b):
        v = np.zeros(4, dtype=np.complex128)
        v[a + 2 * b] = 1
        return v
    return [np.outer(ket(0, 0), ket(0, 0)), np.outer(ket(1, 1), ket(1, 1)),
            np.outer(ket(1, 0), ket(1, 0)), np.outer(ket(1, 0), ket(0, 1))]


def depol2(p):
    """eq. (depol2): (1-p) rho + p/15 sum over the 15 non-identity two-qubit
    Pauli products.  The operators follow the order in which the equation
    writes its terms (which fixes which operator a trajectory's uniform
    draws): the identity, sigma_i for sigma = X, Y, Z, then sigma_j, then
    sigma_i sigma'_j with sigma the outer index."""
    terms = ([(0, 0)] + [(a, 0) for a in (1, 2, 3)] + [(0, b) for b in (1, 2, 3)]
             + [(a, b) for a in (1, 2, 3) for b in (1, 2, 3)])
    return [math.sqrt((1 - p) if (a, b) == (0, 0) else p / 15) * on2(PAULIS[a], PAULIS[b])
            for a, b in terms]


def deph1(p):
    """eq. (deph1): (1-p) rho + p Z rho Z."""
    return [math.sqrt(1 - p) * I2, math.sqrt(p) * Z]


def deph2(p):
    """eq. (deph2): (1-p) rho + p/3 (Z_i rho Z_i + Z_j rho Z_j + Z_iZ_j rho Z_iZ_j)."""
    return [math.sqrt(1 - p) * on2(I2, I2), math.sqrt(p / 3) * on2(Z, I2),
            math.sqrt(p / 3) * on2(I2, Z), math.sqrt(p / 3) * on2(Z, Z)]


def amp(p):
    """eq. (damp): {[[1,0],[0,sqrt(1-p)]], [[0,sqrt(p)],[0,0]]}."""
    return [np.array([[1, 0], [0, math.sqrt(1 - p)]], dtype=np.complex128),
            np.array([[0, math.sqrt(p)], [0, 0]], dtype=np.complex128)]


def gamp(p, gamma):
    """eq. (gdamp): generalised amplitude damping towards p|0><0| + (1-p)|1><1|."""
    a = math.sqrt(p)
    b = math.sqrt(1 - p)
    return [a * np.array([[1, 0], [0, math.sqrt(1 - gamma)]], dtype=np.complex128),
            a * np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128),
            b * np.array([[math.sqrt(1 - gamma), 0], [0, 1]], dtype=np.complex128),
            b * np.array([[0, 0], [math.sqrt(gamma), 0]], dtype=np.complex128)]


def bitflip1(b):
    """eq. (bf): (1-b) rho + b X rho X."""
    return [math.sqrt(1 - b) * I2, math.sqrt(b) * X]


def bitflip2(b):
    """eq. (bf2): (1-b) rho + b/3 (X_i rho X_i + X_j rho X_j + X_iX_j rho X_iX_j)."""
    return [math.sqrt(1 - b) * on2(I2, I2), math.sqrt(b / 3) * on2(X, I2),
            math.sqrt(b / 3) * on2(I2, X), math.sqrt(b / 3) * on2(X, X)]


def amp_t1(dt, T1):
    """eq. (ampt1): amp(1 - exp(-dt/T1))."""
    return amp(1.0 - math.exp(-dt / T1))


def deph_t2(dt, T2):
    """eq. (depht2): deph(1/2 (1 - exp(-dt/T2)))."""
    return deph1(0.5 * (1.0 - math.exp(-dt / T2)))


def deph_t2s(dt, T2s):
    """eq. (depht2s): deph(1/2 (1 - exp(-(dt/T2*)^2))), the Gaussian T2* decay."""
    return deph1(0.5 * (1.0 - math.exp(-(dt / T2s) ** 2)))


def depol_t1(dt, T1):
    """eq. (depolt1): depol(3/4 (1 - exp(-dt/T1)))."""
    return depol1(0.75 * (1.0 - math.exp(-dt / T1)))


def gamp_t1(p, dt, T1):
    """eq. (gdamp) with gamma(dt) = 1 - exp(-dt/T1): T1 relaxation for a time dt
    towards the thermal state p|0><0| + (1-p)|1><1|."""
    return gamp(p, 1.0 - math.exp(-dt / T1))


CHANNELS = {
    "depol1": depol1, "depol2": depol2, "deph1": deph1, "deph2": deph2,
    "amp": amp, "gamp": gamp, "bitflip1": bitflip1, "bitflip2": bitflip2,
    "amp_t1": amp_t1, "deph_t2": deph_t2, "deph_t2s": deph_t2s, "depol_t1": depol_t1,
    "gamp_t1": gamp_t1, "parity_decay": parity_decay,
}


def build(op):
    """(kind, qubits, params) -> ("matrix", M) or ("kraus", [K...])."""
    kind, qubits, params = op
    if kind == "kraus":
        return "kraus", [np.asarray(K, dtype=np.complex128) for K in params]
    if kind in CHANNELS:
        return "kraus", CHANNELS[kind](*params)
    return "matrix", gate_matrix(kind, params)
