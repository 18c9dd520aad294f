"""Seeded op-stream generators for the five workloads.

An op is a tuple ``(kind, qubits, params)``:

* ``kind``   -- a name from :data:`GATE_KINDS` or :data:`CHANNEL_KINDS`,
* ``qubits`` -- tuple of target qubits; ``qubits[0]`` is the least significant
  bit of the op's matrix index,
* ``params`` -- tuple of floats (angles in radians, times in microseconds,
  probabilities), or for the test-only kinds ``"matrix"`` / ``"kraus"`` a
  tuple holding complex numpy arrays.

Only random draws and circuit layout happen here.  Turning a parameter into a
matrix (a rotation, ``1 - exp(-dt/T1)`` for a damping probability, a
normalised quaternion for an SU(2) gate) is left to the consumer, so the
oracle and the GPU path each do it with their own code.

Seeds follow ``SEED_BASE + k`` for workload k (0-based).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

SEED_BASE = 2306073420

Op = Tuple[str, Tuple[int, ...], tuple]

# Unitary kinds and their parameter lists.
GATE_KINDS = {
    "rx": ("theta",), "ry": ("theta",), "rz": ("theta",),
    "h": (), "x": (), "y": (), "z": (),
    "su2": ("g0", "g1", "g2", "g3"),      # 4 raw Gaussian draws (a quaternion)
    "cz": (), "cphase": ("theta",), "xx": ("theta",), "zz": ("alpha",),
    "rabi": ("Omega", "phi", "Delta", "t"), "offres": ("Omega", "Delta", "t"), "crz": ("alpha",),
    "matrix": ("M",),                       # explicit 2^k x 2^k matrix (tests)
}
# Channel kinds and their parameter lists.
CHANNEL_KINDS = {
    "depol1": ("p",), "depol2": ("p",), "deph1": ("p",), "deph2": ("p",),
    "amp": ("p",), "bitflip1": ("b",), "bitflip2": ("b",),
    "amp_t1": ("dt", "T1"), "deph_t2": ("dt", "T2"), "deph_t2s": ("dt", "T2s"), "depol_t1": ("dt", "T1"),
    "gamp": ("p", "gamma"), "gamp_t1": ("p", "dt", "T1"), "parity_decay": (),
    "kraus": ("Ks",),                       # explicit Kraus list (tests)
}


def count_gates(ops: Sequence[Op]) -> int:
    """Number of unitary gates in an op stream (crosstalk ``zz`` included)."""
    return sum(1 for k, _, _ in ops if k in GATE_KINDS)


def _c1_noise(q, p_depol, dt, T1, T2):
    return [("depol1", (q,), (p_depol,)),
            ("amp_t1", (q,), (dt, T1)),
            ("deph_t2", (q,), (dt, T2))]


def _line_circuit(rng, n, n_gates, p_depol, dt, T1, T2) -> List[Op]:
    """Gates drawn uniformly from {Rx, Ry, Rz, CZ} on a line of n qubits;
    after each gate every touched qubit gets depol1 -> amp(T1) -> deph(T2)."""
    ops: List[Op] = []
    for _ in range(n_gates):
        g = int(rng.integers(0, 4))
        if g < 3:
            q = int(rng.integers(0, n))
            th = float(rng.uniform(0.0, 2.0 * math.pi))
            ops.append((("rx", "ry", "rz")[g], (q,), (th,)))
            ops += _c1_noise(q, p_depol, dt, T1, T2)
        else:
            a = int(rng.integers(0, n - 1))
            ops.append(("cz", (a, a + 1), ()))
            for q in (a, a + 1):
                ops += _c1_noise(q, p_depol, dt, T1, T2)
    return ops


def c1_line_circuit(n: int = 6, n_gates: int = 200, seed: int = SEED_BASE + 0) -> List[Op]:
    """6-qubit line, 200 random gates, depol 1e-3, T1=100us, T2=50us, 50 ns gates."""
    rng = np.random.default_rng(seed)
    return _line_circuit(rng, n, n_gates, 1e-3, 0.05, 100.0, 50.0)


def grid_edges(rows: int, cols: int):
    """Edges of a rows x cols grid (q = cols*row + col) split into the three
    matchings used cyclically: horizontal-even, horizontal-odd, vertical."""
    h_even, h_odd, vert = [], [], []
    for r in range(rows):
        for c in range(cols - 1):
            e = (cols * r + c, cols * r + c + 1)
            (h_even if c % 2 == 0 else h_odd).append(e)
    for r in range(rows - 1):
        for c in range(cols):
            vert.append((cols * r + c, cols * (r + 1) + c))
    return [h_even, h_odd, vert]


def c2_grid_circuit(rows: int = 2, cols: int = 7, n_gates: int = 2000,
                    seed: int = SEED_BASE + 1, T1: float = 100.0, T2: float = 50.0,
                    p2: float = 5e-3, zz_alpha: float = 0.01,
                    dt_1q: float = 0.05, dt_2q: float = 0.5) -> List[Op]:
    """Layered grid circuit: a Haar SU(2) layer on every qubit alternates with a
    CZ layer on the next matching; depol2 after each CZ, ZZ crosstalk on the
    idle edges of a CZ layer, amp(T1) and deph(T2) on all qubits at the end of
    every layer.  Stops at exactly ``n_gates`` SU(2)/CZ gates (crosstalk ZZ is
    not counted)."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    matchings = grid_edges(rows, cols)
    all_edges = [e for m in matchings for e in m]
    ops: List[Op] = []
    done = 0
    layer = 0
    while done < n_gates:
        if layer % 2 == 0:
            take = min(n, n_gates - done)
            for q in range(take):
                g = rng.standard_normal(4)
                ops.append(("su2", (q,), tuple(float(x) for x in g)))
            done += take
            dt = dt_1q
        else:
            active = matchings[(layer // 2) % len(matchings)]
            take = min(len(active), n_gates - done)
            for (a, b) in active[:take]:
                ops.append(("cz", (a, b), ()))
                ops.append(("depol2", (a, b), (p2,)))
            done += take
            act = set(active)
            for e in all_edges:
                if e not in act:
                    ops.append(("zz", e, (zz_alpha,)))
            dt = dt_2q
        for q in range(n):
            ops.append(("amp_t1", (q,), (dt, T1)))
            ops.append(("deph_t2", (q,), (dt, T2)))
        layer += 1
    return ops


def c3_all_to_all_circuit(n: int = 16, n_gates: int = 500, seed: int = SEED_BASE + 2,
                          p2: float = 1e-2, p_deph: float = 1e-3) -> List[Op]:
    """Each layer: XX(theta), theta ~ U[0, pi/2], on a uniform random perfect
    matching (depol2 after each), then Rz or Ry (fair coin) with a uniform angle
    on every qubit, then deph1 on every qubit.  Exactly ``n_gates`` gates."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    done = 0
    while done < n_gates:
        perm = rng.permutation(n)
        pairs = [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]
        for (a, b) in pairs[: n_gates - done]:
            th = float(rng.uniform(0.0, math.pi / 2))
            ops.append(("xx", (a, b), (th,)))
            ops.append(("depol2", (a, b), (p2,)))
            done += 1
        for q in range(n):
            if done >= n_gates:
                break
            kind = "rz" if rng.integers(0, 2) == 0 else "ry"
            ops.append((kind, (q,), (float(rng.uniform(0.0, 2 * math.pi)),)))
            done += 1
        for q in range(n):
            ops.append(("deph1", (q,), (p_deph,)))
    return ops


def c4_batch_instances(n_inst: int = 4096, seed: int = SEED_BASE + 3,
                       n_range=(3, 10), ops_range=(100, 400)):
    """Batch of independent line circuits of uneven size with their own noise
    parameters.  Returns a list of dicts ``{n, ops, T1, T2, p, seed}``.

    T1 ~ U[20, 200] us, T2 ~ U[10, T1] us, p ~ log-uniform on [1e-4, 1e-2]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        n_gates = int(rng.integers(ops_range[0], ops_range[1] + 1))
        T1 = float(rng.uniform(20.0, 200.0))
        T2 = float(rng.uniform(10.0, T1))
        p = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        irng = np.random.default_rng(seed + 1 + i)
        ops = _line_circuit(irng, n, n_gates, p, 0.05, T1, T2)
        out.append({"n": n, "ops": ops, "T1": T1, "T2": T2, "p": p,
                    "n_gates": n_gates})
    return out


C5_N = 10
C5_LAYERS = 4
C5_PARAM_NAMES = ("T1", "T2", "p1", "p2", "t1q", "t2q", "zz_alpha", "readout_b")
C5_PARAM_RANGES = ((20.0, 200.0), (10.0, None), (1e-4, 1e-2), (1e-4, 1e-2),
                   (0.02, 0.1), (0.2, 0.8), (0.0, 0.02), (0.0, 0.1))


def c5_ansatz_circuit(dev: Sequence[float], angles: Sequence[float],
                      n: int = C5_N, layers: int = C5_LAYERS) -> List[Op]:
    """Fixed hardware-efficient ansatz with device noise.

    Layer l: Ry(a[4l]) on even qubits, Ry(a[4l+1]) on odd, Rz(a[4l+2]) on even,
    Rz(a[4l+3]) on odd, then CZ bricks (0,1),(2,3),... and (1,2),(3,4),...
    Noise: after every 1q gate depol1(p1), amp(t1q, T1), deph(t1q, T2); after
    every CZ depol2(p2) then amp/deph(t2q) on both qubits; ZZ(alpha) on every
    line edge idle during a brick; a bit flip (readout_b) on every qubit at the
    end, before the read-out."""
    T1, T2, p1, p2, t1q, t2q, alpha, b = (float(x) for x in dev)
    ops: List[Op] = []
    edges = [(i, i + 1) for i in range(n - 1)]
    for l in range(layers):
        for k, kind in enumerate(("ry", "ry", "rz", "rz")):
            th = float(angles[4 * l + k])
            for q in range(k % 2, n, 2):
                ops.append((kind, (q,), (th,)))
                ops.append(("depol1", (q,), (p1,)))
                ops.append(("amp_t1", (q,), (t1q, T1)))
                ops.append(("deph_t2", (q,), (t1q, T2)))
        for start in (0, 1):
            brick = [(a, a + 1) for a in range(start, n - 1, 2)]
            for (a, c) in brick:
                ops.append(("cz", (a, c), ()))
                ops.append(("depol2", (a, c), (p2,)))
                for q in (a, c):
                    ops.append(("amp_t1", (q,), (t2q, T1)))
                    ops.append(("deph_t2", (q,), (t2q, T2)))
            if alpha != 0.0:
                bs = set(brick)
                for e in edges:
                    if e not in bs:
                        ops.append(("zz", e, (alpha,)))
    for q in range(n):
        ops.append(("bitflip1", (q,), (b,)))
    return ops


# slots of the concatenated parameter vector [dev (8), angles (4 * layers)]
_C5_T1, _C5_T2, _C5_P1, _C5_P2, _C5_T1Q, _C5_T2Q, _C5_ALPHA, _C5_B = range(8)


def c5_structure(n: int = C5_N, layers: int = C5_LAYERS):
    """The op sequence of ``c5_ansatz_circuit`` as ``(kind, qubits, slots)``:
    ``slots`` index the concatenated vector ``[dev (8), angles (4*layers)]``
    for each of the op's parameters.  ZZ crosstalk ops are always present
    (ZZ with alpha = 0 is the identity), so one structure serves every
    parameter setting."""
    out = []
    edges = [(i, i + 1) for i in range(n - 1)]
    for l in range(layers):
        for k, kind in enumerate(("ry", "ry", "rz", "rz")):
            for q in range(k % 2, n, 2):
                out.append((kind, (q,), (8 + 4 * l + k,)))
                out.append(("depol1", (q,), (_C5_P1,)))
                out.append(("amp_t1", (q,), (_C5_T1Q, _C5_T1)))
                out.append(("deph_t2", (q,), (_C5_T1Q, _C5_T2)))
        for start in (0, 1):
            brick = [(a, a + 1) for a in range(start, n - 1, 2)]
            for (a, c) in brick:
                out.append(("cz", (a, c), ()))
                out.append(("depol2", (a, c), (_C5_P2,)))
                for q in (a, c):
                    out.append(("amp_t1", (q,), (_C5_T2Q, _C5_T1)))
                    out.append(("deph_t2", (q,), (_C5_T2Q, _C5_T2)))
            bs = set(brick)
            for e in edges:
                if e not in bs:
                    out.append(("zz", e, (_C5_ALPHA,)))
    for q in range(n):
        out.append(("bitflip1", (q,), (_C5_B,)))
    return out


def c5_params(structure, dev: np.ndarray, angles: np.ndarray) -> np.ndarray:
    """Per-op parameters ``[count, n_ops, 4]`` of ``count`` settings: each op's
    slots gathered from ``[dev, angles]`` (unused entries 0)."""
    v = np.concatenate([np.atleast_2d(dev), np.atleast_2d(angles)], axis=1)
    idx = np.full((len(structure), 4), -1, dtype=np.int64)
    for i, (_, _, slots) in enumerate(structure):
        idx[i, :len(slots)] = slots
    out = v[:, np.maximum(idx, 0)]
    out[:, idx < 0] = 0.0
    return np.ascontiguousarray(out)


def c5_draw_samples(count: int, seed: int = SEED_BASE + 4, n_angles: int = 4 * C5_LAYERS):
    """Draw ``count`` (device parameters, circuit angles) pairs.

    Returns ``(dev[count, 8], angles[count, 16])`` as float64 arrays with the
    raw physical values (angles in [0, 2 pi))."""
    rng = np.random.default_rng(seed)
    dev = np.empty((count, 8))
    dev[:, 0] = rng.uniform(20.0, 200.0, count)
    u = rng.uniform(0.0, 1.0, count)
    dev[:, 1] = 10.0 + u * (dev[:, 0] - 10.0)          # T2 ~ U[10, T1]
    dev[:, 2] = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), count))
    dev[:, 3] = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), count))
    dev[:, 4] = rng.uniform(0.02, 0.1, count)
    dev[:, 5] = rng.uniform(0.2, 0.8, count)
    dev[:, 6] = rng.uniform(0.0, 0.02, count)
    dev[:, 7] = rng.uniform(0.0, 0.1, count)
    angles = rng.uniform(0.0, 2 * math.pi, (count, n_angles))
    return dev, angles


def random_matrix_ops(n: int, count: int, seed: int, kraus: bool = True,
                      max_k: int = 2, scale: float = 1.0) -> List[Op]:
    """Random op stream on n qubits made of explicit matrices: Gaussian complex
    2^k x 2^k matrices ("matrix", applied as M rho M^dagger) and, if ``kraus``,
    lists of 1..4 Gaussian Kraus matrices.  Entries are (N(0,1)+iN(0,1)) times
    ``scale / sqrt(2 d m)`` for m matrices of size d, so that the sum of
    K^dagger K is the identity on average; no single map is trace preserving,
    which the emulator must handle as well.  Targets are distinct and in
    random order."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for _ in range(count):
        k = int(rng.integers(1, min(max_k, n) + 1))
        tg = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        d = 2 ** k
        if kraus and rng.integers(0, 2) == 1:
            nk = int(rng.integers(1, 5))
            s = scale / math.sqrt(2.0 * d * nk)
            Ks = tuple((rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * s
                       for _ in range(nk))
            ops.append(("kraus", tg, Ks))
        else:
            s = scale / math.sqrt(2.0 * d)
            M = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * s
            ops.append(("matrix", tg, (M,)))
    return ops
