"""Noise insertion for a virtual device -- TEST INFRASTRUCTURE (the oracle).

Only tests use this module.  It maps an ideal gate list to the noisy op
stream a device specification prescribes (Sec. 2: active noise after each
gate, passive noise on idle qubits for the duration of the slowest operation
of their automatically scheduled parallel batch; Sec. 3.4 crosstalk; Sec. 3.5
passive T1/T2 decay, eqs. ampt1, depolt1, depht2 and depht2s; Sec. 8: T1
relaxation towards the thermal state, eq. gdamp, the static ZZ coupling of
transmons, and the read-out model; App. C: errors scaled by the rotation
angle).

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
* Gate kinds without a specification take no time and add no noise.  A
  specification for a gate kind on a particular set of qubits (App. C: per-
  qubit rotation fidelities, per-pair two-qubit gates) replaces the kind's
  for gates on exactly those qubits, in any order; the kind's angle scaling
  applies to it.
* T1 decay is amp_t1, or gamp_t1(p0, dt, T1) when the qubit's thermal ground
  population p0 is below 1 (relaxation towards the state it is initialised
  in, eq. thermalstate), or depol_t1 when that form is chosen; T2 decay is
  deph_t2 or, when chosen, the Gaussian deph_t2s.
* Static ZZ coupling beta (phase per unit time) acts on its pair for the
  whole duration of every batch, as one ZZ(beta dt) emitted after the
  idle-edge crosstalk, except in batches with a two-qubit gate on that very
  pair (the paper: a driven coupler gate removes it).
* Angle scaling (App. C) multiplies a gate's active noise probabilities,
  and if asked its duration, by |theta|/pi for its first parameter theta.
* Off-resonant driving (Sec. 3.3, used by the silicon device of Sec. 7):
  with per-qubit Rabi frequencies Omega_q and qubit frequencies w_q (both
  angular, per unit time), a one-qubit gate of duration t > 0 on a qubit q
  with Omega_q > 0 drives q, and every qubit j that is passive in the batch
  (not a target of any of its gates) receives eq. off_resonant with
  (Omega_q, w_j - w_q, t).  These ops follow the batch's gates and active
  noise, grouped by driving gate in input order and, within one, by
  ascending j; they precede crosstalk and passive decay.  Several drives in
  one batch act one after another.
* Serial devices (Sec. 7): every gate forms a batch of its own, in input
  order.
* Exchange crosstalk (Sec. 7) on listed edges (c, t): the conditional Z
  rotation of eq. weak_dephasing, control c, on edges whose two qubits are
  passive in the batch.  A two-qubit gate of angle theta (its first
  parameter, pi for a gate without one) on listed edge i gives every other
  edge j crz(on[i][j] theta / pi), by gate in input order and then by edge;
  a batch without two-qubit gates gives edge j crz(off[j]).  Zero angles are
  left out.  These ops follow the off-resonant ones.
* Parity read-out (Sec. 7, eq. projmeas) of a pair: bitflip2(b) (eq. bf2),
  T1 and T2 decay for the read-out time on every other qubit (ascending),
  then the decay map parity_decay on the pair, before the parity projection
  (eq. m); bitflip2(b) after it.
* Read-out form "bitflip1" (the trapped ions, Sec. 4): a symmetric bit flip
  eps (eq. bf) on each measured qubit before the projection, nothing after
  it; qubits not measured idle for the measurement time (T1, T2).
* Read-out (Sec. 8): T1 decay for the measurement time, then
  depolarising noise eps, before the projection; depolarising noise eps
  after it.  Qubits not measured idle for the measurement time (T1, T2).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple


class Device:
    def __init__(self, n: int):
        self.n = n
        self.gates: Dict[str, Tuple[float, float, float]] = {}   # kind -> (duration, p_depol, p_deph)
        self.gates_on: Dict[Tuple[str, Tuple[int, ...]], Tuple[float, float, float]] = {}
        self.scaling: Dict[str, Tuple[bool, bool]] = {}          # kind -> (noise, duration)
        self.T1 = [0.0] * n
        self.T2 = [0.0] * n
        self.p0 = [1.0] * n
        self.t1_form, self.t2_form = "amp_t1", "deph_t2"
        self.edges: List[Tuple[int, int]] = []
        self.alpha = 0.0
        self.static_zz: List[Tuple[int, int, float]] = []
        self.t_meas = 0.0
        self.eps = [0.0] * n
        self.rabi: List[float] = []      # off-resonant driving: Omega_q and w_q
        self.freq: List[float] = []
        self.serial = False
        self.par_t, self.par_b = 0.0, 0.0           # parity read-out
        self.readout_form = "depol1"
        self.xe_edges: List[Tuple[int, int]] = []   # exchange crosstalk
        self.xe_on: List[List[float]] = []
        self.xe_off: List[float] = []

    def set_gate_on(self, kind: str, qubits, duration: float, p_depol: float = 0.0, p_deph: float = 0.0):
        self.gates_on[(kind, tuple(sorted(qubits)))] = (duration, p_depol, p_deph)

    def set_angle_scaling(self, kind: str, noise: bool = True, duration: bool = False):
        self.scaling[kind] = (noise, duration)

    def set_thermal(self, p0: Sequence[float]):
        self.p0 = list(p0)

    def set_passive_forms(self, t1: str = "amp_t1", t2: str = "deph_t2"):
        self.t1_form, self.t2_form = t1, t2

    def set_static_zz(self, edges, beta):
        self.static_zz = [(int(a), int(b), float(x)) for (a, b), x in zip(edges, beta)]

    def set_readout(self, t_meas: float, eps: Sequence[float]):
        self.t_meas, self.eps = t_meas, list(eps)

    def set_parity_readout(self, t_meas: float, b: float):
        self.par_t, self.par_b = t_meas, b

    def set_readout_form(self, kind: str = "depol1"):
        self.readout_form = kind

    def set_serial(self, serial: bool = True):
        self.serial = bool(serial)

    def set_exchange_crosstalk(self, edges, on, off):
        self.xe_edges = [tuple(int(x) for x in e) for e in edges]
        self.xe_on = [list(r) for r in on]
        self.xe_off = list(off)

    def set_off_resonant(self, rabi: Sequence[float], freq: Sequence[float]):
        self.rabi, self.freq = list(rabi), list(freq)

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


def _t1(dev: Device, q: int, dt: float) -> List[tuple]:
    if dev.T1[q] <= 0 or dt <= 0:
        return []
    if dev.t1_form == "depol_t1":
        return [("depol_t1", (q,), (dt, dev.T1[q]))]
    if dev.p0[q] < 1:
        return [("gamp_t1", (q,), (dev.p0[q], dt, dev.T1[q]))]
    return [("amp_t1", (q,), (dt, dev.T1[q]))]


def _t2(dev: Device, q: int, dt: float) -> List[tuple]:
    if dev.T2[q] <= 0 or dt <= 0:
        return []
    return [(dev.t2_form, (q,), (dt, dev.T2[q]))]


def insert_noise(dev: Device, gates: Sequence) -> List[tuple]:
    out: List[tuple] = []
    batches = [[i] for i in range(len(gates))] if dev.serial else schedule(dev.n, gates)
    for batch in batches:
        spec = []
        for i in batch:
            kind, qs, params = gates[i]
            d, pd, pq = dev.gates_on.get((kind, tuple(sorted(qs))), dev.gates.get(kind, (0.0, 0.0, 0.0)))
            scale_noise, scale_dur = dev.scaling.get(kind, (False, False))
            f = abs(params[0]) / math.pi if (scale_noise or scale_dur) else 1.0
            if scale_noise:
                pd, pq = pd * f, pq * f
                if pd > 1 or pq > 1:
                    raise ValueError("angle-scaled noise probability above 1")
            if scale_dur:
                d = d * f
            spec.append((d, pd, pq))
        dur = max(s[0] for s in spec)
        busy = {}
        pairs = set()
        for i, (d, pd, pq) in zip(batch, spec):
            kind, qs, params = gates[i]
            out.append((kind, tuple(qs), tuple(params)))
            k = len(qs)
            if k == 2:
                pairs.add(frozenset(qs))
            if pd > 0:
                out.append(("depol1" if k == 1 else "depol2", tuple(qs), (pd,)))
            if pq > 0:
                out.append(("deph1" if k == 1 else "deph2", tuple(qs), (pq,)))
            for q in qs:
                busy[q] = d
        if dev.rabi:
            for i, (d, _, _) in zip(batch, spec):
                qs = gates[i][1]
                if len(qs) != 1 or d <= 0 or dev.rabi[qs[0]] <= 0:
                    continue
                q = qs[0]
                for j in range(dev.n):
                    if j not in busy:
                        out.append(("offres", (j,), (dev.rabi[q], dev.freq[j] - dev.freq[q], d)))
        def passive_edge(e):
            return e[0] not in busy and e[1] not in busy
        for i in batch:
            kind, qs, params = gates[i]
            if len(qs) != 2 or frozenset(qs) not in [frozenset(e) for e in dev.xe_edges]:
                continue
            a = [frozenset(e) for e in dev.xe_edges].index(frozenset(qs))
            theta = params[0] if params else math.pi
            for j, e in enumerate(dev.xe_edges):
                alpha = dev.xe_on[a][j] * theta / math.pi
                if j != a and alpha != 0 and passive_edge(e):
                    out.append(("crz", e, (alpha,)))
        if not pairs:
            for j, e in enumerate(dev.xe_edges):
                if dev.xe_off[j] != 0 and passive_edge(e):
                    out.append(("crz", e, (dev.xe_off[j],)))
        if pairs and dev.alpha != 0:
            for a, b in dev.edges:
                if a not in busy and b not in busy:
                    out.append(("zz", (a, b), (dev.alpha,)))
        if dur > 0:
            for a, b, beta in dev.static_zz:
                if beta != 0 and frozenset((a, b)) not in pairs:
                    out.append(("zz", (a, b), (beta * dur,)))
        for q in range(dev.n):
            idle = dur - busy.get(q, 0.0)
            if idle > 0:
                out += _t1(dev, q, idle) + _t2(dev, q, idle)
    return out


def readout_noise(dev: Device, qubits: Sequence[int], stage: int) -> List[tuple]:
    """Noise of the read-out model around a projective measurement of
    ``qubits``: stage 0 before it, stage 1 after it."""
    if len(set(qubits)) != len(qubits):
        raise ValueError("duplicate qubit")
    out: List[tuple] = []
    for q in qubits:
        if dev.readout_form == "bitflip1":
            if stage == 0 and dev.eps[q] > 0:
                out.append(("bitflip1", (q,), (dev.eps[q],)))
            continue
        if stage == 0:
            out += _t1(dev, q, dev.t_meas)
        if dev.eps[q] > 0:
            out.append(("depol1", (q,), (dev.eps[q],)))
    if stage == 0:
        for q in range(dev.n):
            if q not in qubits:
                out += _t1(dev, q, dev.t_meas) + _t2(dev, q, dev.t_meas)
    return out


def parity_readout_noise(dev: Device, q0: int, q1: int, stage: int) -> List[tuple]:
    """Noise of the parity read-out of (q0, q1): stage 0 before the parity
    projection (ending with the read-out's decay map), stage 1 after it."""
    out: List[tuple] = []
    if dev.par_b > 0:
        out.append(("bitflip2", (q0, q1), (dev.par_b,)))
    if stage == 0:
        if dev.par_t > 0:
            for q in range(dev.n):
                if q not in (q0, q1):
                    out += _t1(dev, q, dev.par_t) + _t2(dev, q, dev.par_t)
        out.append(("parity_decay", (q0, q1), ()))
    return out
