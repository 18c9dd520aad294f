"""Monte Carlo state-vector trajectories -- TEST INFRASTRUCTURE (the oracle).

Only tests, the smoke check and the benchmark's CPU baseline use this module;
the library never does.

The paper (Sec. 2, "The virtual quantum device package", where it compares
the state-vector and density-matrix representations) describes the alternative to the density matrix: each decoherence channel is
replaced, in one sample, by a single operator drawn from its Kraus map and
applied to a state vector; expected values are averaged over many samples.

Readings taken here (the paper gives no more detail):

* Operator K_i of a channel {K_i} is drawn with probability
  w_i / W, where w_i = ||K_i psi||^2 and W = sum_i w_i (the Born rule of the
  unravelling, which makes the average of |psi><psi| equal to the channel's
  action on the density matrix).  The state becomes K_i psi / sqrt(w_i).
* Each channel consumes one uniform variate u in [0, 1), in op order.  The
  drawn index is the smallest i whose running sum w_0 + ... + w_i exceeds
  u * W (sums taken left to right); if rounding leaves none, the last i with
  w_i > 0.
* Gates act as psi -> M psi and draw nothing.
* A trajectory starts in |0...0>.  Its outputs are <Z_q> = sum_x |psi_x|^2
  (1 - 2 x_q) and the squared norm sum_x |psi_x|^2.

Matrices act on their qubits with qubits[0] as the least significant bit of
the matrix index (the convention of oracle.channels).
"""
from __future__ import annotations

import math
from typing import Iterable, List, Sequence, Tuple

import numpy as np

from . import channels


def _offsets(qubits: Sequence[int]) -> np.ndarray:
    """Basis-index offset of local index l (bit j of l -> qubit qubits[j])."""
    k = len(qubits)
    return np.array([sum(((l >> j) & 1) << q for j, q in enumerate(qubits)) for l in range(1 << k)],
                    dtype=np.int64)


def _bases(n: int, qubits: Sequence[int]) -> np.ndarray:
    """Basis indices whose target bits are all zero."""
    mask = sum(1 << q for q in qubits)
    x = np.arange(1 << n, dtype=np.int64)
    return x[(x & mask) == 0]


def apply_matrix(psi: np.ndarray, qubits: Sequence[int], M: np.ndarray) -> np.ndarray:
    """M acting on the subspace of ``qubits``: for every setting of the other
    bits, the 2^k amplitudes it selects are multiplied by M."""
    n = int(psi.size).bit_length() - 1
    idx = _bases(n, qubits)[:, None] | _offsets(qubits)[None, :]
    out = psi.copy()
    out[idx] = psi[idx] @ np.asarray(M, dtype=np.complex128).T
    return out


def kraus_weights(psi: np.ndarray, qubits: Sequence[int], Ks) -> List[float]:
    """w_i = ||K_i psi||^2."""
    out = []
    for K in Ks:
        phi = apply_matrix(psi, qubits, K)
        out.append(float(np.vdot(phi, phi).real))
    return out


def draw(w: Sequence[float], u: float) -> int:
    """Index drawn by u from weights w (see the module docstring)."""
    W = 0.0
    for x in w:
        W += x
    thr = u * W
    cum = 0.0
    for i, x in enumerate(w):
        cum += x
        if cum > thr:
            return i
    return max(i for i, x in enumerate(w) if x > 0)


def step(psi: np.ndarray, op, u: float = None) -> Tuple[np.ndarray, int, List[float]]:
    """Apply one op.  Gates return (M psi, -1, []); channels need ``u`` and
    return (K_j psi / sqrt(w_j), j, w)."""
    what, payload = channels.build(op)
    qubits = op[1]
    if what == "matrix":
        return apply_matrix(psi, qubits, payload), -1, []
    w = kraus_weights(psi, qubits, payload)
    j = draw(w, u)
    return apply_matrix(psi, qubits, payload[j]) / math.sqrt(w[j]), j, w


def is_channel(op) -> bool:
    return op[0] in channels.CHANNELS or op[0] == "kraus"


def n_channels(ops: Iterable) -> int:
    """Uniform variates one trajectory consumes."""
    return sum(1 for op in ops if is_channel(op))


def initial_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def run(n: int, ops: Sequence, u: Sequence[float]) -> Tuple[np.ndarray, List[int]]:
    """One trajectory: final state and the drawn Kraus index of every channel."""
    need = n_channels(ops)
    if need != len(u):
        raise ValueError("the ops hold %d channels, %d uniforms given" % (need, len(u)))
    psi = initial_state(n)
    drawn = []
    c = 0
    for op in ops:
        if is_channel(op):
            psi, j, _ = step(psi, op, float(u[c]))
            drawn.append(j)
            c += 1
        else:
            psi, _, _ = step(psi, op)
    return psi, drawn


def expec_z(psi: np.ndarray) -> np.ndarray:
    """<Z_q> for every qubit (un-normalised: sum_x |psi_x|^2 (1 - 2 x_q))."""
    n = int(psi.size).bit_length() - 1
    p = np.abs(psi) ** 2
    x = np.arange(psi.size)
    return np.array([np.sum(p * (1 - 2 * ((x >> q) & 1))) for q in range(n)])


def norm2(psi: np.ndarray) -> float:
    return float(np.sum(np.abs(psi) ** 2))


def run_many(n: int, ops: Sequence, U: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Trajectories for the rows of U (T x channels): per-trajectory <Z_q>
    (T x n) and squared norms (T)."""
    Z = np.empty((U.shape[0], n))
    N = np.empty(U.shape[0])
    for t in range(U.shape[0]):
        psi, _ = run(n, ops, U[t])
        Z[t] = expec_z(psi)
        N[t] = norm2(psi)
    return Z, N


def estimate(samples: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Mean over trajectories (axis 0) and its standard error
    (sample standard deviation / sqrt(T))."""
    T = samples.shape[0]
    mean = samples.mean(axis=0)
    if T < 2:
        return mean, np.full_like(mean, np.inf)
    return mean, samples.std(axis=0, ddof=1) / math.sqrt(T)
