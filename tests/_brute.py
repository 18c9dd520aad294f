"""Brute-force density-matrix reference for tiny registers (n <= 4).

Independent of the oracle's C loops: rho is reshaped into a tensor with one
axis per row qubit and one per column qubit, and every operator is contracted
on the target axes with ``np.tensordot``.  Qubit q is axis ``n-1-q`` of the
row block (C order puts the most significant bit first).
"""
from __future__ import annotations

import numpy as np


def _axis(n, q):
    return n - 1 - q


def apply_left(rho, n, targets, M):
    """M_T rho for an operator M on ``targets`` (targets[0] = LSB of M's index)."""
    k = len(targets)
    T = rho.reshape((2,) * (2 * n))
    # M as a tensor: output bits (b_{k-1} ... b_0), input bits likewise
    Mt = M.reshape((2,) * (2 * k))
    # input axes of Mt: k..2k-1 correspond to targets[k-1], ..., targets[0]
    row_axes = [_axis(n, targets[k - 1 - j]) for j in range(k)]
    out = np.tensordot(Mt, T, axes=(list(range(k, 2 * k)), row_axes))
    # out axes: M's output axes first, then remaining T axes in order
    remaining = [a for a in range(2 * n) if a not in row_axes]
    order = [None] * (2 * n)
    for j in range(k):
        order[row_axes[j]] = j
    for i, a in enumerate(remaining):
        order[a] = k + i
    return np.transpose(out, order).reshape(rho.shape)


def apply_op(rho, n, targets, M):
    """M rho M^dagger."""
    left = apply_left(rho, n, targets, M)
    return apply_left(left.conj().T, n, targets, M).conj().T


def apply_kraus(rho, n, targets, Ks):
    return sum(apply_op(rho, n, targets, K) for K in Ks)


def embed(n, targets, M):
    """Full 2^n x 2^n operator for M on ``targets``."""
    return apply_left(np.eye(1 << n, dtype=np.complex128), n, targets, M)


def pauli_string(codes):
    """Full matrix of (x)_q sigma_{codes[q]}, qubit 0 the least significant."""
    P = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]])]
    out = np.array([[1.0 + 0j]])
    for c in codes:                     # qubit q goes to the left of qubits < q
        out = np.kron(P[c], out)
    return out
