"""The library's noise insertion (vqd_device_*) against the oracle
(oracle/device.py): identical op streams for hand-made and random circuits
and device specifications."""
import numpy as np
import pytest

from oracle import device as dv
from tests.test_device_oracle import random_gates, spec4, spec_sc
from workloads import c1_line_circuit, c2_grid_circuit


def same_stream(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x[0] == y[0] and tuple(x[1]) == tuple(y[1]), (x, y)
        assert np.allclose(x[2], y[2], rtol=0, atol=1e-15), (x, y)


def lib_device(vqd, ref: dv.Device):
    d = vqd.Device(ref.n)
    for k, (t, p, q) in ref.gates.items():
        d.set_gate(k, t, p, q)
    d.set_passive(ref.T1, ref.T2)
    d.set_crosstalk(ref.edges, ref.alpha)
    for (k, qs), (t, p, q) in ref.gates_on.items():
        d.set_gate_on(k, qs, t, p, q)
    for k, (noise, dur) in ref.scaling.items():
        d.set_angle_scaling(k, noise, dur)
    d.set_thermal(ref.p0)
    d.set_passive_forms(ref.t1_form, ref.t2_form)
    d.set_static_zz([(a, b) for a, b, _ in ref.static_zz], [x for _, _, x in ref.static_zz])
    d.set_readout(ref.t_meas, ref.eps)
    if ref.rabi:
        d.set_off_resonant(ref.rabi, ref.freq)
    d.set_serial(ref.serial)
    d.set_parity_readout(ref.par_t, ref.par_b)
    d.set_readout_form(ref.readout_form)
    if ref.xe_edges:
        d.set_exchange_crosstalk(ref.xe_edges, ref.xe_on, ref.xe_off)
    return d


def test_hand_example(vqd_host):
    ref = spec4()
    gates = [("h", (0,), ()), ("cz", (0, 1), ()), ("x", (2,), ())]
    same_stream(lib_device(vqd_host, ref).insert_noise(gates), dv.insert_noise(ref, gates))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_circuits_and_devices(vqd_host, seed):
    rng = np.random.default_rng(seed)
    n = 7
    ref = dv.Device(n)
    for k in ("rx", "ry", "rz", "h", "cz"):
        if rng.random() < 0.9:
            ref.set_gate(k, float(rng.choice([0.0, 0.02, 0.05, 0.3])), float(rng.choice([0.0, 1e-3])),
                         float(rng.choice([0.0, 2e-3])))
    T1 = rng.uniform(20, 200, n) * (rng.random(n) < 0.8)
    ref.set_passive(list(T1), list(rng.uniform(10, 100, n) * (rng.random(n) < 0.8)))
    ref.set_crosstalk([(i, i + 1) for i in range(n - 1)], float(rng.choice([0.0, 0.01])))
    gates = random_gates(n, 80, seed)
    same_stream(lib_device(vqd_host, ref).insert_noise(gates), dv.insert_noise(ref, gates))


def test_grid_gates_with_a_superconducting_like_device(vqd_host):
    ideal = [op for op in c2_grid_circuit(rows=2, cols=4, n_gates=120) if op[0] in ("su2", "cz")]
    ref = dv.Device(8)
    ref.set_gate("su2", 0.05, 1e-3, 5e-4)
    ref.set_gate("cz", 0.5, 5e-3, 1e-3)
    ref.set_passive([100.0] * 8, [50.0] * 8)
    ref.set_crosstalk([(a, a + 1) for a in range(7) if a != 3] + [(a, a + 4) for a in range(4)], 0.01)
    same_stream(lib_device(vqd_host, ref).insert_noise(ideal), dv.insert_noise(ref, ideal))


def test_hand_example_with_every_rule(vqd_host):
    ref = spec_sc()
    gates = [("rx", (0,), (np.pi / 2,)), ("cz", (1, 2), ())]
    same_stream(lib_device(vqd_host, ref).insert_noise(gates), dv.insert_noise(ref, gates))


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_random_devices_with_every_rule(vqd_host, seed):
    rng = np.random.default_rng(seed)
    n = 6
    ref = dv.Device(n)
    for k in ("rx", "ry", "rz", "h", "cz"):
        ref.set_gate(k, float(rng.choice([0.0, 0.05, 0.3])), float(rng.choice([0.0, 1e-3])),
                     float(rng.choice([0.0, 2e-3])))
    for k in ("rx", "ry"):
        ref.set_angle_scaling(k, bool(rng.integers(2)), bool(rng.integers(2)))
    for q in range(n):                            # per-qubit rotation specs
        if rng.random() < 0.5:
            ref.set_gate_on("rx", (q,), float(rng.choice([0.03, 0.07])), float(rng.uniform(0, 2e-3)))
    for a in range(n - 1):                        # per-pair CZ specs
        if rng.random() < 0.5:
            ref.set_gate_on("cz", (a + 1, a), float(rng.choice([0.2, 0.4])), float(rng.uniform(0, 1e-2)),
                            float(rng.uniform(0, 1e-2)))
    ref.set_passive(list(rng.uniform(20, 200, n) * (rng.random(n) < 0.8)),
                    list(rng.uniform(10, 100, n) * (rng.random(n) < 0.8)))
    ref.set_thermal(list(np.where(rng.random(n) < 0.5, 1.0, rng.uniform(0.9, 1.0, n))))
    ref.set_passive_forms(str(rng.choice(["amp_t1", "depol_t1"])), str(rng.choice(["deph_t2", "deph_t2s"])))
    ref.set_crosstalk([(i, i + 1) for i in range(n - 1)], 0.01)
    ref.set_static_zz([(i, i + 1) for i in range(n - 1)] + [(0, n - 1)], list(rng.uniform(-0.05, 0.05, n)))
    ref.set_readout(float(rng.uniform(1, 5)), list(rng.uniform(0, 0.05, n) * (rng.random(n) < 0.7)))
    ref.set_off_resonant(list(rng.uniform(1, 10, n) * (rng.random(n) < 0.7)), list(rng.uniform(-50, 50, n)))
    xe = [(i + 1, i) if rng.random() < 0.5 else (i, i + 1) for i in range(n - 1)] + [(0, 2)]
    ref.set_exchange_crosstalk(xe, rng.uniform(0, 0.1, (len(xe), len(xe))) * (rng.random((len(xe), len(xe))) < 0.7),
                               rng.uniform(0, 0.05, len(xe)) * (rng.random(len(xe)) < 0.7))
    ref.set_serial(seed % 2 == 0)
    ref.set_parity_readout(float(rng.uniform(0, 12)), float(rng.uniform(0, 0.1)))
    ref.set_readout_form(["depol1", "bitflip1"][seed % 2])
    gates = random_gates(n, 80, seed)
    lib = lib_device(vqd_host, ref)
    same_stream(lib.insert_noise(gates), dv.insert_noise(ref, gates))
    for qs in ([0], [3, 1], list(range(n)), []):
        for stage in (0, 1):
            same_stream(lib.readout_noise(qs, stage), dv.readout_noise(ref, qs, stage))
    for q0, q1 in ((0, 1), (5, 2)):
        for stage in (0, 1):
            same_stream(lib.parity_readout_noise(q0, q1, stage), dv.parity_readout_noise(ref, q0, q1, stage))


def test_off_resonant_hand_stream(vqd_host):
    ref = dv.Device(3)
    ref.set_gate("rx", 0.1)
    ref.set_gate("ry", 0.3)
    ref.set_off_resonant([2.0, 0.0, 5.0], [10.0, 13.0, 17.0])
    gates = [("rx", (0,), (0.5,)), ("rz", (1,), (0.2,)), ("cz", (1, 2), ()), ("ry", (2,), (1.0,)),
             ("rx", (1,), (0.3,))]
    lib = lib_device(vqd_host, ref)
    same_stream(lib.insert_noise(gates), dv.insert_noise(ref, gates))
    lib.set_off_resonant(None)                      # off again: no offres ops
    assert all(k != "offres" for k, _, _ in lib.insert_noise(gates))
    with pytest.raises(vqd_host.VQDError):
        lib.set_off_resonant([1.0, -1.0, 0.0], [0.0, 0.0, 0.0])
    with pytest.raises(vqd_host.VQDError):
        lib.set_off_resonant([1.0, 1.0, 0.0], [0.0, float("nan"), 0.0])
    with pytest.raises(vqd_host.VQDError):
        lib.set_exchange_crosstalk([(0, 1), (1, 0)], np.zeros((2, 2)), [0.0, 0.0])     # repeated edge
    with pytest.raises(vqd_host.VQDError):
        lib.set_exchange_crosstalk([(0, 3)], [[0.0]], [0.0])                         # no qubit 3
    with pytest.raises(vqd_host.VQDError):
        lib.set_exchange_crosstalk([(0, 1)], [[float("inf")]], [0.0])
    lib.set_exchange_crosstalk([], [], [])                                           # off
    with pytest.raises(vqd_host.VQDError):
        lib.set_readout_form("amp")
    with pytest.raises(vqd_host.VQDError):
        lib.set_parity_readout(10.0, 0.8)                                            # b > 0.75
    with pytest.raises(vqd_host.VQDError):
        lib.set_parity_readout(-1.0, 0.1)
    with pytest.raises(vqd_host.VQDError):
        lib.parity_readout_noise(0, 0, 0)
    with pytest.raises(vqd_host.VQDError):
        lib.parity_readout_noise(0, 1, 2)


def test_zz_strength(vqd_host):
    from oracle.params import zz_strength
    for args in ((4.0, -400.0, 296.7, 298.6), (1.5, 200.0, 297.4, 297.2), (0.0, 10.0, 1.0, 2.0)):
        assert abs(vqd_host.zz_crosstalk_strength(*args) - zz_strength(*args)) <= 1e-15
    with pytest.raises(vqd_host.VQDError):
        vqd_host.zz_crosstalk_strength(1.0, 5.0, 1.0, 5.0)        # Delta - alpha_t = 0


def test_errors(vqd_host):
    v = vqd_host
    with pytest.raises(v.VQDError):
        v.Device(0)
    d = v.Device(3)
    with pytest.raises(v.VQDError):
        d.set_gate("depol1", 0.1)                # a channel is not a gate
    with pytest.raises(v.VQDError):
        d.set_gate("cz", -1.0)
    with pytest.raises(v.VQDError):
        d.set_crosstalk([(0, 3)], 0.1)
    with pytest.raises(v.VQDError):
        d.insert_noise([("cz", (0, 0), ())])
    assert d.insert_noise([]) == []
    with pytest.raises(v.VQDError):
        d.set_angle_scaling("h")                     # no angle
    with pytest.raises(v.VQDError):
        d.set_gate_on("cz", (0,), 0.1)              # two targets needed
    with pytest.raises(v.VQDError):
        d.set_gate_on("cz", (0, 0), 0.1)
    with pytest.raises(v.VQDError):
        d.set_gate_on("depol1", (0,), 0.1)
    with pytest.raises(v.VQDError):
        d.set_thermal([1.0, 1.2, 0.5])
    with pytest.raises(v.VQDError):
        d.set_passive_forms("deph_t2", "deph_t2")
    with pytest.raises(v.VQDError):
        d.set_static_zz([(0, 0)], [0.1])
    with pytest.raises(v.VQDError):
        d.set_readout(-1.0, [0.0] * 3)
    d.set_readout(1.0, [0.1] * 3)
    with pytest.raises(v.VQDError):
        d.readout_noise([1, 1], 0)
    with pytest.raises(v.VQDError):
        d.readout_noise([0], 2)
    d.set_gate("rx", 0.1, 0.5)
    d.set_angle_scaling("rx")
    with pytest.raises(v.VQDError):                  # 0.5 * 3 > 1
        d.insert_noise([("rx", (0,), (3 * np.pi,))])
