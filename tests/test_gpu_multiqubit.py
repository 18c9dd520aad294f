"""The neutral-atom multi-qubit operations of Sec. 6 on the density-matrix
path against the oracle: the multi-controlled C_Q Z_p and the controlled
multi-Z C_p Z_Q (diagonal gates on up to four qubits, with the global
phase i of their definitions), and the leakage map M = (x)_j M_j,
M_j = diag(1, sqrt(1 - alpha)), a single-operator trace-decreasing map that
the library applies as its one-qubit factors."""
import math
import sys

import numpy as np
import pytest

from oracle.core import OracleDM
from oracle.emulator import emulate
from workloads import random_tp_ops

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cqz(k):
    """C_Q Z_p on targets (Q..., p): phase -1 on |1...1>, times i."""
    d = np.ones(1 << (k + 1), dtype=complex)
    d[-1] = -1
    return 1j * np.diag(d)


def cpzq(k):
    """C_p Z_Q on targets (p, Q...): Z on every Q qubit when p = 1, times i."""
    D = 1 << (k + 1)
    d = np.ones(D, dtype=complex)
    for x in range(D):
        if x & 1:
            d[x] = (-1) ** bin(x >> 1).count("1")
    return 1j * np.diag(d)


def start(gpu_lib, n, seed):
    ops = random_tp_ops(n, 2 * n, seed=seed, max_k=2)
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, ops).compile().run(dm)
    return dm, emulate(n, ops)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_multi_controlled_z(gpu_lib, k):
    n = 6
    say("C_Q Z_p and C_p Z_Q, |Q| = %d" % k)
    tg = tuple(range(n - 1, n - 2 - k, -1))           # high qubits, descending
    for M in (cqz(k), cpzq(k)):
        dm, ref = start(gpu_lib, n, 11 + k)
        gpu_lib.Program(n, [("matrix", tg, (M,))]).compile().run(dm)
        ref.apply_matrix(list(tg), M)
        assert np.abs(dm.to_numpy() - ref.to_vectorised()).max() <= TOL


def test_leakage_map_as_one_qubit_factors(gpu_lib):
    n, alpha = 6, 0.2
    Q = (0, 2, 3, 5, 1)
    say("leakage map on %d qubits" % len(Q))
    Mj = np.diag([1.0, math.sqrt(1 - alpha)]).astype(complex)
    dm, ref = start(gpu_lib, n, 3)
    gpu_lib.Program(n, [("kraus", (q,), (Mj,)) for q in Q]).compile().run(dm)
    full = np.array([[1.0]], dtype=complex)
    for _ in Q:
        full = np.kron(Mj, full)                  # Q[0] the least significant bit
    ref.apply_matrix(list(Q), full)
    assert np.abs(dm.to_numpy() - ref.to_vectorised()).max() <= TOL
    assert dm.trace().real < 1.0                 # trace decreasing
