"""Noise insertion for a virtual device -- TEST INFRASTRUCTURE (the oracle).

Only tests use this module.  It maps an ideal gate list to the noisy op
stream a device specification prescribes (Sec. 2: active noise after each
gate, passive noise on idle qubits for the duration of the slowest operation
of their automatically scheduled parallel batch; Sec. 3.4 crosstalk; Sec. 3.5
passive T1/T2 decay, eqs. ampt1 and depht2).

Readings (the paper describes the behaviour, not a procedure):

* Scheduling is as-soon-as-possible: a gate joins the batch after the last
  batch that uses any of its qubits.  A batch lasts as long as its slowest
  gate.
* A batch is emitted as: each of its gates in input order, each followed by
  its active noise on its qubits (depolarising, then dephasing; one- or
  two-qubit forms by the gate's size); then, if the batch holds a two-qubit
  gate, ZZ crosstalk on every listed edge whose two qubits are both idle in
  the batch; then, for every qubit in ascending order, passive amp_t1 and
  deph_t2 for the time it is idle in the batch (the whole batch for an idle
  qubit, the batch minus the gate for a qubit whose gate is shorter).
* Operations with no effect are left out: zero probabilities, zero idle
  time, a disabled T1 or T2 (<= 0), zero crosstalk phase.
* Gate kinds without a specification take no time and add no noise.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple


class Device:
    def __init__(self, n: int):
        self.n = n
        self.gates: Dict[str, Tuple[float, float, float]] = {}   # kind -> (duration, p_depol, p_deph)
        self.T1 = [0.0] * n
        self.T2 = [0.0] * n
        self.edges: List[Tuple[int, int]] = []
        self.alpha = 0.0

    def set_gate(self, kind: str, duration: float, p_depol: float = 0.0, p_deph: float = 0.0):
        self.gates[kind] = (duration, p_depol, p_deph)

    def set_passive(self, T1: Sequence[float], T2: Sequence[float]):
        self.T1, self.T2 = list(T1), list(T2)

    def set_crosstalk(self, edges, alpha: float):
        self.edges, self.alpha = [tuple(e) for e in edges], alpha


def schedule(n: int, gates: Sequence) -> List[List[int]]:
    """Batches of gate indices (as soon as possible)."""
    last = [-1] * n
    batches: List[List[int]] = []
    for i, (_, qs, _) in enumerate(gates):
        b = 1 + max(last[q] for q in qs)
        while len(batches) <= b:
            batches.append([])
        batches[b].append(i)
        for q in qs:
            last[q] = b
    return batches


def insert_noise(dev: Device, gates: Sequence) -> List[tuple]:
    out: List[tuple] = []
    for batch in schedule(dev.n, gates):
        spec = [dev.gates.get(gates[i][0], (0.0, 0.0, 0.0)) for i in batch]
        dur = max(s[0] for s in spec)
        busy = {}
        two_qubit = False
        for i, (d, pd, pq) in zip(batch, spec):
            kind, qs, params = gates[i]
            out.append((kind, tuple(qs), tuple(params)))
            k = len(qs)
            two_qubit = two_qubit or k == 2
            if pd > 0:
                out.append(("depol1" if k == 1 else "depol2", tuple(qs), (pd,)))
            if pq > 0:
                out.append(("deph1" if k == 1 else "deph2", tuple(qs), (pq,)))
            for q in qs:
                busy[q] = d
        if two_qubit and dev.alpha != 0:
            for a, b in dev.edges:
                if a not in busy and b not in busy:
                    out.append(("zz", (a, b), (dev.alpha,)))
        for q in range(dev.n):
            idle = dur - busy.get(q, 0.0)
            if idle > 0:
                if dev.T1[q] > 0:
                    out.append(("amp_t1", (q,), (idle, dev.T1[q])))
                if dev.T2[q] > 0:
                    out.append(("deph_t2", (q,), (idle, dev.T2[q])))
    return out
