"""Pins of the noise-insertion oracle (oracle/device.py): a hand-scheduled
example, time bookkeeping, per-qubit gate order, and a noise-free device
reproducing the ideal circuit's state."""
import numpy as np
import pytest

from oracle import device as dv
from oracle.emulator import emulate
from workloads import c1_line_circuit


def spec4():
    d = dv.Device(4)
    d.set_gate("h", 0.05, p_depol=0.001)
    d.set_gate("x", 0.03)
    d.set_gate("cz", 0.2, p_depol=0.01, p_deph=0.002)
    d.set_passive([100.0] * 4, [50.0] * 4)
    d.set_crosstalk([(2, 3), (1, 2)], 0.01)
    return d


def test_hand_scheduled_example():
    gates = [("h", (0,), ()), ("cz", (0, 1), ()), ("x", (2,), ())]
    got = dv.insert_noise(spec4(), gates)
    expect = [
        # batch 0: H on 0 and X on 2 (0.05 us, the H)
        ("h", (0,), ()), ("depol1", (0,), (0.001,)), ("x", (2,), ()),
        ("amp_t1", (1,), (0.05, 100.0)), ("deph_t2", (1,), (0.05, 50.0)),
        ("amp_t1", (2,), (0.05 - 0.03, 100.0)), ("deph_t2", (2,), (0.05 - 0.03, 50.0)),
        ("amp_t1", (3,), (0.05, 100.0)), ("deph_t2", (3,), (0.05, 50.0)),
        # batch 1: CZ on (0, 1) (0.2 us); edge (2, 3) idle, edge (1, 2) not
        ("cz", (0, 1), ()), ("depol2", (0, 1), (0.01,)), ("deph2", (0, 1), (0.002,)),
        ("zz", (2, 3), (0.01,)),
        ("amp_t1", (2,), (0.2, 100.0)), ("deph_t2", (2,), (0.2, 50.0)),
        ("amp_t1", (3,), (0.2, 100.0)), ("deph_t2", (3,), (0.2, 50.0)),
    ]
    assert len(got) == len(expect)
    for g, e in zip(got, expect):
        assert g[0] == e[0] and g[1] == e[1] and np.allclose(g[2], e[2], rtol=0, atol=1e-15)


def random_gates(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = rng.integers(0, 5)
        if k < 3:
            out.append((("rx", "ry", "rz")[k], (int(rng.integers(n)),), (float(rng.uniform(0, 6)),)))
        elif k == 3:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append(("cz", (a, b), ()))
        else:
            out.append(("h", (int(rng.integers(n)),), ()))
    return out


def test_time_bookkeeping_and_order():
    n = 5
    d = dv.Device(n)
    for k, t in (("rx", 0.04), ("ry", 0.04), ("rz", 0.01), ("h", 0.03), ("cz", 0.3)):
        d.set_gate(k, t, p_depol=1e-3)
    d.set_passive([80.0] * n, [40.0] * n)
    gates = random_gates(n, 60, 3)
    out = dv.insert_noise(d, gates)
    batches = dv.schedule(n, gates)
    total = sum(max(d.gates[gates[i][0]][0] for i in b) for b in batches)
    for q in range(n):
        idle = sum(p[0] for k, qs, p in out if k == "amp_t1" and qs == (q,))
        busy = sum(d.gates[k][0] for k, qs, _ in out if k in d.gates and q in qs)
        assert abs(idle + busy - total) <= 1e-12
        assert [g for g in out if g[0] in d.gates and q in g[1]] == [g for g in gates if q in g[1]]


def test_noise_free_device_reproduces_the_ideal_state():
    n = 4
    gates = [op for op in c1_line_circuit(n=n, n_gates=40) if op[0] in ("rx", "ry", "rz", "cz")]
    d = dv.Device(n)
    for k in ("rx", "ry", "rz"):
        d.set_gate(k, 0.05)
    d.set_gate("cz", 0.2)
    out = dv.insert_noise(d, gates)
    assert sorted(map(str, out)) == sorted(map(str, gates))
    assert np.abs(emulate(n, out).R - emulate(n, gates).R).max() <= 1e-13
