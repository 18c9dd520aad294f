"""Device presets (vqd_device_preset) against devices the test builds on the
oracle from the paper's printed tables (tests/golden/device_tables.json,
App. C) with the oracle's own conversions: the ZZ coupling formula of Sec. 8
(oracle.params.zz_strength) and the App. B fidelity inversion by bisection
(oracle.params.severity).  The two sides share only the printed numbers."""
import json
import math
import os

import numpy as np
import pytest

from oracle import device as dv
from oracle.params import severity, zz_strength
from tests.test_device_cpu import same_stream
from tests.test_device_oracle import random_gates

HERE = os.path.dirname(os.path.abspath(__file__))
TABLES = json.load(open(os.path.join(HERE, "golden", "device_tables.json")))


def oracle_superconducting():
    t = TABLES["superconducting"]
    n = t["QubitNum"]
    d = dv.Device(n)
    for k in ("rx", "ry", "h", "x", "y", "su2"):
        d.set_gate(k, t["DurRxRy"])
    for k in ("cz", "cphase", "xx", "zz"):
        d.set_gate(k, t["DurZZ"])
    d.set_passive(t["T1"], t["T2"])
    p0 = [1 - x for x in t["ExcitedInit"]]
    d.set_thermal(p0)
    f, a = t["QubitFreq"], t["Anharmonicity"]
    edges = [(c, q) for c, q, _ in t["ExchangeCoupling"]]
    beta = [2 * math.pi * zz_strength(J, f[c] - f[q], a[c], a[q]) for c, q, J in t["ExchangeCoupling"]]
    d.set_static_zz(edges, beta)
    d.set_readout(t["DurMeas"], [1 - x for x in t["FidRead"]])
    return d, p0


def oracle_trapped_ion():
    t = TABLES["trapped_ion"]
    n = sum(k for _, k in t["Nodes"])
    d = dv.Device(n)
    x1 = t["EFSingleXY"][0] / sum(t["EFSingleXY"])
    x2 = t["EFCZ"][0] / sum(t["EFCZ"])
    p1, q1 = severity(t["FidSingleXY"], 1, x1)
    p2, q2 = severity(t["FidCZ"], 2, x2)
    t_pi = 1 / (2 * t["RabiFreq"])
    for k in ("rx", "ry"):
        d.set_gate(k, t_pi, p1, q1)
        d.set_angle_scaling(k, noise=True, duration=True)
    for k in ("h", "x", "y"):
        d.set_gate(k, t_pi, p1, q1)
    d.set_gate("cz", 1 / (2 * t["FreqCZ"]), p2, q2)
    d.set_passive([t["T1"]] * n, [t["T2s"]] * n)
    d.set_passive_forms("amp_t1", "deph_t2s")
    d.set_readout(t["DurRead"], [t["BFProb"]] * n)
    d.set_readout_form("bitflip1")
    return d, [t["FidInit"]] * n


def oracle_silicon():
    t = TABLES["silicon"]
    n = t["QubitNum"]
    d = dv.Device(n)
    x1 = t["EFSingleXY"][0] / sum(t["EFSingleXY"])
    x2 = t["EFCZ"][0] / sum(t["EFCZ"])
    for q in range(n):
        p, s = severity(t["FidSingleXY"][q], 1, x1)
        for k in ("rx", "ry", "h", "x", "y"):
            d.set_gate_on(k, (q,), 1 / (2 * t["RabiFreq"][q]), p, s)
    for k in ("rx", "ry", "cphase"):
        d.set_angle_scaling(k, noise=True, duration=True)
    edges = [(q, q + 1) for q in range(n - 1)]
    for e, (a, b) in enumerate(edges):
        p, s = severity(t["FidCZ"][e], 2, x2)
        for k in ("cz", "cphase"):
            d.set_gate_on(k, (a, b), 1 / (2 * t["FreqCZ"][e]), p, s)
    d.set_passive([t["T1"]] * n, t["T2"])
    d.set_passive_forms("depol_t1", "deph_t2")
    d.set_off_resonant([2 * math.pi * f for f in t["RabiFreq"]], [2 * math.pi * f for f in t["QubitFreq"]])
    d.set_exchange_crosstalk(edges, t["ExchangeRotOn"], t["ExchangeRotOff"])
    d.set_serial(True)
    d.set_parity_readout(t["DurRead"], 1 - t["FidRead"])
    return d, [1.0] * n


def si_gates(n, count, seed):
    """x and y rotations, Hadamards, CZ and CPhase on the line of spins."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(0, 5))
        if k < 2:
            out.append((("rx", "ry")[k], (int(rng.integers(n)),), (float(rng.uniform(-3, 3)),)))
        elif k == 2:
            out.append(("h", (int(rng.integers(n)),), ()))
        else:
            a = int(rng.integers(n - 1))
            out.append(("cz", (a, a + 1), ()) if k == 3 else ("cphase", (a + 1, a), (float(rng.uniform(-3, 3)),)))
    return out


def close_stream(a, b, tol):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x[0] == y[0] and tuple(x[1]) == tuple(y[1]), (x, y)
        assert np.allclose(x[2], y[2], rtol=tol, atol=1e-15), (x, y)


def sc_gates(n, count, seed):
    """Rotations, Hadamards and CZ on the coupled pairs of the transmon grid."""
    rng = np.random.default_rng(seed)
    pairs = [(c, q) for c, q, _ in TABLES["superconducting"]["ExchangeCoupling"]]
    out = []
    for _ in range(count):
        k = rng.integers(0, 4)
        if k < 2:
            out.append((("ry", "rz")[k], (int(rng.integers(n)),), (float(rng.uniform(-3, 3)),)))
        elif k == 2:
            out.append(("h", (int(rng.integers(n)),), ()))
        else:
            out.append(("cz", pairs[int(rng.integers(len(pairs)))], ()))
    return out


def test_superconducting_preset(vqd_host):
    lib, p0 = vqd_host.Device.preset("superconducting")
    ref, rp0 = oracle_superconducting()
    assert lib.n == ref.n == 6
    assert np.abs(p0 - rp0).max() <= 1e-15
    gates = sc_gates(6, 60, 11)
    # the coupling goes through the same formula on both sides: only rounding
    close_stream(lib.insert_noise(gates), dv.insert_noise(ref, gates), 1e-13)
    kinds = {k for k, _, _ in lib.insert_noise(gates)}
    assert {"gamp_t1", "deph_t2", "zz"} <= kinds and "amp_t1" not in kinds
    for qs in ([0], [5, 2], list(range(6))):
        for stage in (0, 1):
            same_stream(lib.readout_noise(qs, stage), dv.readout_noise(ref, qs, stage))


def test_trapped_ion_preset(vqd_host):
    lib, p0 = vqd_host.Device.preset("trapped_ion")
    ref, rp0 = oracle_trapped_ion()
    assert lib.n == ref.n == 8
    assert np.abs(p0 - rp0).max() == 0
    gates = random_gates(8, 60, 12)
    # closed-form root (library) against bisection (oracle)
    close_stream(lib.insert_noise(gates), dv.insert_noise(ref, gates), 1e-9)
    for qs in ([0], [7, 2]):
        for stage in (0, 1):
            same_stream(lib.readout_noise(qs, stage), dv.readout_noise(ref, qs, stage))
    assert [k for k, _, _ in lib.readout_noise([3], 0)][0] == "bitflip1" and lib.readout_noise([3], 1) == []


def test_silicon_preset(vqd_host):
    lib, p0 = vqd_host.Device.preset("silicon")
    ref, rp0 = oracle_silicon()
    assert lib.n == ref.n == 6
    assert np.abs(p0 - rp0).max() == 0
    gates = si_gates(6, 60, 13)
    got = lib.insert_noise(gates)
    close_stream(got, dv.insert_noise(ref, gates), 1e-9)
    kinds = {k for k, _, _ in got}
    assert {"offres", "crz", "deph1", "deph2", "depol_t1", "deph_t2"} <= kinds and "depol1" not in kinds
    for q0, q1 in ((0, 1), (4, 5)):
        for stage in (0, 1):
            close_stream(lib.parity_readout_noise(q0, q1, stage), dv.parity_readout_noise(ref, q0, q1, stage), 1e-15)


def test_superconducting_coupling_values():
    """Spot values of the Sec. 8 formula on the tabulated pair (Q0, Q1):
    J = 4, Delta = -400, alpha = 296.7 and 298.6 MHz."""
    b = 16 * (1 / (-400 - 298.6) - 1 / (-400 + 296.7))
    assert abs(zz_strength(4, -400, 296.7, 298.6) - b) <= 1e-15
    assert 0.13 < b < 0.14                          # about 0.132 MHz


def test_unknown_preset(vqd_host):
    with pytest.raises(KeyError):
        vqd_host.Device.preset("nv_centre")
    import ctypes
    h = ctypes.c_void_p()
    assert vqd_host.lib().vqd_device_preset(99, ctypes.byref(h), None) != 0
