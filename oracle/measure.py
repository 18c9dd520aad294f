"""Measurement on the density-matrix oracle -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the benchmark's CPU baseline use this module.

* Projective measurement in the computational basis of one qubit (the
  readout of the trapped-ion, NV-centre and neutral-atom devices, Secs. 4-6):
  outcome m in {0, 1} with weight w_m = Re Tr(P_m rho), P_m = |m><m| on the
  qubit, and post-measurement state P_m rho P_m / w_m.
* Parity measurement of two qubits, eq. (m): outcome "0" for the odd-parity
  projector |01><01| + |10><10| and "1" for the even-parity projector
  |00><00| + |11><11|, in that order.
* Shot sampling (the 2000 simulated measurements of Sec. 6): basis states x
  drawn from the diagonal probabilities p_x = Re rho_xx.

Readings (the paper gives no sampling procedure):

* Every draw takes one caller-supplied uniform u in [0, 1) and the rule of
  the trajectory oracle (oracle.trajectories.draw): the smallest index whose
  running sum of weights, taken in index order, exceeds u W, W the sum of
  all weights; the last positive weight if rounding leaves none.
* Outcome weights are the projectors' traces, not renormalised: a state of
  trace t != 1 draws with w_m / t.
* Diagonal probabilities below zero (rounding residue of a zero population)
  count as zero when sampling.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .core import OracleDM
from .trajectories import draw


def _projector(n_bits: int, keep: Sequence[int]) -> np.ndarray:
    P = np.zeros((1 << n_bits, 1 << n_bits), dtype=np.complex128)
    for x in keep:
        P[x, x] = 1.0
    return P


def _measure(dm: OracleDM, qubits: Sequence[int], projectors: List[np.ndarray], u: float
             ) -> Tuple[int, List[float]]:
    diag = np.real(np.diag(dm.R))
    x = np.arange(diag.size)
    local = np.zeros(diag.size, dtype=np.int64)
    for j, q in enumerate(qubits):
        local |= ((x >> q) & 1) << j
    w = [float(sum(diag[local == l].sum() for l in range(P.shape[0]) if P[l, l] != 0)) for P in projectors]
    m = draw(w, u)
    dm.apply_matrix(list(qubits), projectors[m])
    dm.R /= w[m]
    return m, w


def measure_z(dm: OracleDM, q: int, u: float) -> Tuple[int, List[float]]:
    """Projective Z measurement of qubit q; collapses dm in place and returns
    (outcome, [w_0, w_1])."""
    return _measure(dm, [q], [_projector(1, [0]), _projector(1, [1])], u)


def measure_parity(dm: OracleDM, q0: int, q1: int, u: float) -> Tuple[int, List[float]]:
    """Parity measurement of eq. (m) on (q0, q1); outcome 0 = odd parity,
    1 = even parity.  Collapses dm in place and returns (outcome, [w_0, w_1])."""
    odd = _projector(2, [1, 2])          # |01> and |10> (index b(q0) + 2 b(q1))
    even = _projector(2, [0, 3])
    return _measure(dm, [q0, q1], [odd, even], u)


def sample(probs: np.ndarray, U: Sequence[float]) -> np.ndarray:
    """Basis states drawn from `probs` (negative entries count as zero), one
    per uniform: the draw rule above, with the running sums formed once
    (left to right, as the rule forms them) and searched for each uniform."""
    p = np.maximum(np.asarray(probs, dtype=np.float64), 0.0)
    cum = np.cumsum(p)                   # sequential running sums, cum[-1] = W
    thr = np.asarray(U, dtype=np.float64) * cum[-1]
    idx = np.searchsorted(cum, thr, side="right")     # first index with cum > thr
    last = int(np.nonzero(p > 0)[0][-1])
    return np.where(idx < p.size, idx, last).astype(np.int64)
