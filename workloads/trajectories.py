"""Seeded inputs of the Monte Carlo trajectory mode.

* the uniform variates a batch of trajectories consumes (one per channel per
  trajectory, in op order), drawn here and handed to both the oracle and the
  library;
* random unitary gates and random trace-preserving Kraus maps for tests;
* the trajectory benchmark circuit (the layered grid circuit on a 2x6 grid).
"""
from __future__ import annotations

from typing import List

import numpy as np

from .circuits import SEED_BASE, Op, c2_grid_circuit

TRAJ_SEED = SEED_BASE + 13


def uniforms(T: int, n_channels: int, seed: int = TRAJ_SEED) -> np.ndarray:
    """(T, n_channels) float64 variates in [0, 1), trajectory-major."""
    return np.random.default_rng(seed).random((T, n_channels))


def _haar_like(rng, d):
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def random_tp_ops(n: int, count: int, seed: int, max_k: int = 2, p_channel: float = 0.5) -> List[Op]:
    """Random op stream of unitary gates ("matrix") and trace-preserving Kraus
    maps ("kraus", 1..4 operators cut from a random isometry), on distinct
    targets in random order."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for _ in range(count):
        k = int(rng.integers(1, min(max_k, n) + 1))
        tg = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        d = 2 ** k
        if rng.random() < p_channel:
            m = int(rng.integers(1, 5))
            A = rng.standard_normal((d * m, d)) + 1j * rng.standard_normal((d * m, d))
            V, _ = np.linalg.qr(A)                     # d*m x d with orthonormal columns
            ops.append(("kraus", tg, tuple(V[i * d:(i + 1) * d, :].copy() for i in range(m))))
        else:
            ops.append(("matrix", tg, (_haar_like(rng, d),)))
    return ops


def traj_grid_circuit(n_gates: int = 2000) -> List[Op]:
    """The layered grid circuit (SU(2) layers, CZ + depol2, ZZ crosstalk,
    T1/T2 damping every layer) on a 2x6 grid: 12 qubits."""
    return c2_grid_circuit(rows=2, cols=6, n_gates=n_gates)


def damped_layer_circuit(n: int, layers: int, seed: int, dt_t1: float = 0.25, dt_t2: float = 0.3) -> List[Op]:
    """Layers of seeded SU(2) gates, a CZ chain, then T1 and T2 noise on every
    qubit with dt/T1 and dt/T2 large enough that damping jumps are common
    (a stress case for the runs of damping draws)."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for _ in range(layers):
        for q in range(n):
            ops.append(("su2", (q,), tuple(rng.standard_normal(4))))
        for q in range(0, n - 1, 2):
            ops.append(("cz", (q, q + 1), ()))
        for q in range(n):
            ops.append(("amp_t1", (q,), (dt_t1, 1.0)))
            ops.append(("deph_t2", (q,), (dt_t2, 1.0)))
    return ops
