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


def spec_sc():
    """A device with every optional rule on: thermal relaxation, Gaussian
    dephasing, static ZZ coupling, angle-scaled noise and durations."""
    d = dv.Device(3)
    d.set_gate("rx", 0.1, p_depol=0.02, p_deph=0.01)
    d.set_gate("cz", 0.4)
    d.set_angle_scaling("rx", noise=True, duration=True)
    d.set_passive([60.0, 80.0, 0.0], [30.0, 40.0, 20.0])
    d.set_thermal([0.97, 1.0, 0.9])
    d.set_passive_forms("amp_t1", "deph_t2s")
    d.set_static_zz([(0, 1), (1, 2)], [0.03, -0.02])
    return d


def test_hand_example_with_every_rule():
    pi = np.pi
    gates = [("rx", (0,), (pi / 2,)), ("cz", (1, 2), ())]
    got = dv.insert_noise(spec_sc(), gates)
    expect = [
        # one batch: Rx(pi/2) on 0 (0.05 us, noise halved), CZ on (1, 2) (0.4 us)
        ("rx", (0,), (pi / 2,)), ("depol1", (0,), (0.01,)), ("deph1", (0,), (0.005,)),
        ("cz", (1, 2), ()),
        ("zz", (0, 1), (0.03 * 0.4,)),                    # (1, 2) carries the CZ
        ("gamp_t1", (0,), (0.97, 0.35, 60.0)), ("deph_t2s", (0,), (0.35, 30.0)),
    ]
    assert len(got) == len(expect), got
    for g, e in zip(got, expect):
        assert g[0] == e[0] and g[1] == e[1] and np.allclose(g[2], e[2], rtol=0, atol=1e-15), (g, e)
    with pytest.raises(ValueError):                   # |theta|/pi = 60 pushes 0.02 above 1
        dv.insert_noise(spec_sc(), [("rx", (0,), (60 * pi,))])


def test_idle_qubit_relaxes_towards_its_thermal_state():
    """Qubit 1 is flipped and then idles while qubit 0 runs 39 more X gates:
    its excited population decays as e^{-t/T1} towards 1 - p0, t the idle
    time (the first batch holds both qubits' X)."""
    d = dv.Device(2)
    d.set_gate("x", 0.25)
    d.set_passive([0.0, 3.0], [0.0, 0.0])
    d.set_thermal([1.0, 0.8])
    gates = [("x", (1,), ())] + [("x", (0,), ())] * 40
    dm = emulate(2, dv.insert_noise(d, gates))
    t = 39 * 0.25
    p1 = dm.R[2, 2].real + dm.R[3, 3].real           # qubit 1 excited
    assert abs(p1 - ((1 - 0.8) + 0.8 * np.exp(-t / 3.0))) <= 1e-13


@pytest.mark.parametrize("b", [0, 1])
def test_static_coupling_accumulates_phase(b):
    """|+> on qubit 0, |b> on qubit 1, gates only on qubit 2: the coupling
    beta on (0, 1) rotates qubit 0 by exp(-i (-1)^b beta t Z), so <X_0> =
    cos(2 beta t) and <Y_0> = (-1)^b sin(2 beta t)."""
    d = dv.Device(3)
    d.set_gate("h", 0.1)
    d.set_gate("z", 0.3)
    beta = 0.37
    d.set_static_zz([(0, 1)], [beta])
    prep = [("h", (0,), ())] + ([("x", (1,), ())] if b else [])
    gates = [("z", (2,), ())] * 7
    dm = emulate(3, prep + dv.insert_noise(d, gates))
    t = 7 * 0.3
    assert abs(dm.expec_pauli([1, 0, 0]).real - np.cos(2 * beta * t)) <= 1e-13
    assert abs(dm.expec_pauli([2, 0, 0]).real - (-1) ** b * np.sin(2 * beta * t)) <= 1e-13


def test_readout_flip_probability():
    """|1> read out after T1 decay for t_M and depolarising eps: the outcome
    is 1 with probability e^{-t/T1} (1 - 2eps/3) + (1 - e^{-t/T1}) 2eps/3."""
    d = dv.Device(2)
    d.set_passive([25.0, 40.0], [10.0, 10.0])
    d.set_readout(5.0, [0.06, 0.0])
    pre = dv.readout_noise(d, [0], 0)
    assert [k for k, _, _ in pre] == ["amp_t1", "depol1", "amp_t1", "deph_t2"]
    dm = emulate(2, [("x", (0,), ())] + pre)
    e = np.exp(-5.0 / 25.0)
    p1 = dm.R[1, 1].real + dm.R[3, 3].real
    assert abs(p1 - (e * (1 - 0.04) + (1 - e) * 0.04)) <= 1e-14
    assert dv.readout_noise(d, [0], 1) == [("depol1", (0,), (0.06,))]
    assert dv.readout_noise(d, [1], 1) == []


def test_zz_strength_closed_forms():
    """Sec. 8's coupling: zero without coupling, the same whichever transmon
    is called control, and 2 alpha J^2 / (Delta^2 - alpha^2) for equal
    anharmonicities."""
    from oracle.params import zz_strength
    J, fc, ft, ac, at = 4.0, 4500.0, 4900.0, 296.7, 298.6
    assert zz_strength(0.0, fc - ft, ac, at) == 0.0
    assert abs(zz_strength(J, fc - ft, ac, at) - zz_strength(J, ft - fc, at, ac)) <= 1e-15
    D, a = -400.0, 297.0
    assert abs(zz_strength(J, D, a, a) - 2 * a * J * J / (D * D - a * a)) <= 1e-15


def test_per_target_specifications():
    """A pair's own CZ specification and a qubit's own rotation noise replace
    the kind's; angle scaling applies to both."""
    d = dv.Device(3)
    d.set_gate("cz", 0.2, p_depol=0.01)
    d.set_gate_on("cz", (2, 1), 0.3, p_depol=0.02, p_deph=0.03)
    d.set_gate("rx", 0.1, p_depol=0.004)
    d.set_gate_on("rx", (2,), 0.1, p_depol=0.008)
    d.set_angle_scaling("rx", noise=True)
    gates = [("cz", (1, 2), ()), ("rx", (0,), (np.pi / 2,)), ("rx", (2,), (np.pi,)), ("cz", (0, 1), ())]
    got = dv.insert_noise(d, gates)
    expect = [
        # batch 0: CZ(1, 2) with the pair's spec (0.3 us), Rx(pi/2) on 0 (0.05 us)
        ("cz", (1, 2), ()), ("depol2", (1, 2), (0.02,)), ("deph2", (1, 2), (0.03,)),
        ("rx", (0,), (np.pi / 2,)), ("depol1", (0,), (0.002,)),
        # batch 1: Rx(pi) on 2 with qubit 2's own noise, CZ(0, 1) with the kind's
        ("rx", (2,), (np.pi,)), ("depol1", (2,), (0.008,)),
        ("cz", (0, 1), ()), ("depol2", (0, 1), (0.01,)),
    ]
    assert len(got) == len(expect), got
    for g, e in zip(got, expect):
        assert g[0] == e[0] and g[1] == e[1] and np.allclose(g[2], e[2], rtol=0, atol=1e-15), (g, e)


def test_off_resonant_hand_stream():
    """Sec. 3.3 by hand: a driven one-qubit gate gives every passive qubit of
    its batch eq. off_resonant with the driver's Rabi frequency, the
    bystander's frequency difference and the gate's duration; targets of
    other gates in the batch, undriven qubits and gates of no duration
    drive nothing."""
    d = dv.Device(3)
    d.set_gate("rx", 0.1)
    d.set_gate("ry", 0.3)
    d.set_off_resonant([2.0, 0.0, 5.0], [10.0, 13.0, 17.0])
    gates = [("rx", (0,), (0.5,)), ("rz", (1,), (0.2,)),    # batch 1: 2 is passive
             ("cz", (1, 2), ()),                             # batch 2: no drive
             ("ry", (2,), (1.0,)),                           # batch 3: 0 is passive
             ("rx", (1,), (0.3,))]                           # batch 3: Rabi 0 on qubit 1
    want = [("rx", (0,), (0.5,)), ("rz", (1,), (0.2,)), ("offres", (2,), (2.0, 7.0, 0.1)),
            ("cz", (1, 2), ()),
            ("ry", (2,), (1.0,)), ("rx", (1,), (0.3,)), ("offres", (0,), (5.0, -7.0, 0.3))]
    got = dv.insert_noise(d, gates)
    assert [(k, tuple(q), tuple(p)) for k, q, p in got] == want


@pytest.mark.parametrize("delta", [0.0, 1.5, -4.0, 40.0])
def test_off_resonant_bystander_follows_rabi_formula(delta):
    """A resonant pi pulse on qubit 0 (duration pi / Omega) excites a passive
    qubit detuned by Delta with Rabi's probability
    (Omega/W)^2 sin^2(W t / 2), W = sqrt(Omega^2 + Delta^2)."""
    omega = 3.0
    t = np.pi / omega
    d = dv.Device(2)
    d.set_gate("rx", t)
    d.set_off_resonant([omega, 0.0], [1.0, 1.0 + delta])
    dm = emulate(2, dv.insert_noise(d, [("rx", (0,), (np.pi,))]))
    w = np.hypot(omega, delta)
    p1 = dm.R[2, 2].real + dm.R[3, 3].real             # qubit 1 excited
    assert abs(p1 - (omega / w) ** 2 * np.sin(w * t / 2) ** 2) <= 1e-14
    p0 = dm.R[1, 1].real + dm.R[3, 3].real             # qubit 0: the pi pulse itself
    assert abs(p0 - 1.0) <= 1e-14


@pytest.mark.parametrize("alpha", [0.3, -1.7, 2.9])
def test_crz_is_a_target_rotation_and_a_zz_phase(alpha):
    """eq. (weak_dephasing) against two independent forms: the projector sum
    |0><0| (x) I + |1><1| (x) exp(-i alpha Z / 2) built with scipy's expm,
    and the product Rz_t(alpha / 2) exp(+i alpha/4 Z(x)Z) of the two
    crosstalk forms of Sec. 3.4."""
    from scipy.linalg import expm
    from oracle import channels as ch
    P0, P1 = np.diag([1.0, 0.0]), np.diag([0.0, 1.0])
    want = np.kron(np.eye(2), P0) + np.kron(expm(-0.5j * alpha * ch.Z), P1)   # control = low bit
    U = ch.gate_matrix("crz", (alpha,))
    assert np.abs(U - want).max() < 1e-15
    rz_t = np.kron(ch.gate_matrix("rz", (alpha / 2,)), np.eye(2))
    assert np.abs(U - rz_t @ ch.gate_matrix("zz", (-alpha / 4,))).max() < 1e-15


def test_serial_device_runs_one_gate_per_batch():
    """Two gates on different qubits share a batch as soon as possible, and
    run one after another on a serial device: the idle qubit then waits for
    each of them."""
    d = dv.Device(2)
    d.set_gate("x", 0.5)
    d.set_passive([0.0, 0.0], [10.0, 10.0])
    gates = [("x", (0,), ()), ("x", (1,), ())]
    assert [k for k, _, _ in dv.insert_noise(d, gates)] == ["x", "x"]
    d.set_serial(True)
    want = [("x", (0,), ()), ("deph_t2", (1,), (0.5, 10.0)), ("x", (1,), ()), ("deph_t2", (0,), (0.5, 10.0))]
    assert [(k, tuple(q), tuple(p)) for k, q, p in dv.insert_noise(d, gates)] == want


def test_exchange_crosstalk_hand_stream():
    """Sec. 7 by hand on a line of four qubits, edges (0,1), (1,2), (2,3):
    a CPhase(theta) on edge 0 turns the passive edge 2 by on[0][2] theta/pi
    (edge 1 touches an active qubit); a batch of one-qubit gates gives every
    passive edge its off value; zero entries emit nothing."""
    d = dv.Device(4)
    d.set_serial(True)
    on = [[0.0, 0.1, 0.2], [0.3, 0.0, 0.0], [0.5, 0.6, 0.0]]
    d.set_exchange_crosstalk([(0, 1), (1, 2), (3, 2)], on, [0.01, 0.0, 0.03])
    gates = [("cphase", (1, 0), (np.pi / 2,)), ("rx", (0,), (0.4,)), ("cz", (2, 3), ())]
    want = [("cphase", (1, 0), (np.pi / 2,)), ("crz", (3, 2), (0.1,)),
            ("rx", (0,), (0.4,)), ("crz", (3, 2), (0.03,)),
            ("cz", (2, 3), ()), ("crz", (0, 1), (0.5,))]
    got = [(k, tuple(q), tuple(p)) for k, q, p in dv.insert_noise(d, gates)]
    assert len(got) == len(want)
    for g, w in zip(got, want):
        assert g[:2] == w[:2] and np.allclose(g[2], w[2], rtol=0, atol=1e-15), (g, w)


def test_parity_readout_hand_stream():
    """Sec. 7 by hand: bit flips on the measured pair, the other qubits'
    passive decay for the read-out time, the decay map before the parity
    projection; bit flips again after it."""
    d = dv.Device(3)
    d.set_passive([0.0, 0.0, 50.0], [0.0, 0.0, 20.0])
    d.set_passive_forms("depol_t1", "deph_t2")
    d.set_parity_readout(10.0, 0.01)
    got0 = [(k, tuple(q), tuple(p)) for k, q, p in dv.parity_readout_noise(d, 1, 0, 0)]
    assert got0 == [("bitflip2", (1, 0), (0.01,)), ("depol_t1", (2,), (10.0, 50.0)),
                    ("deph_t2", (2,), (10.0, 20.0)), ("parity_decay", (1, 0), ())]
    got1 = [(k, tuple(q), tuple(p)) for k, q, p in dv.parity_readout_noise(d, 1, 0, 1)]
    assert got1 == [("bitflip2", (1, 0), (0.01,))]


def test_bit_flip_readout_form():
    """Sec. 4: the ions' read-out error is a symmetric bit flip before the
    projection.  The stream holds it for the measured ion and idle decay for
    the others; a prepared |1> then reads 0 with probability b exactly."""
    from oracle import measure as om
    d = dv.Device(2)
    d.set_passive([0.0, 40.0], [0.0, 30.0])
    d.set_readout(50.0, [0.001, 0.002])
    d.set_readout_form("bitflip1")
    got = [(k, tuple(q), tuple(p)) for k, q, p in dv.readout_noise(d, [0], 0)]
    assert got == [("bitflip1", (0,), (0.001,)), ("amp_t1", (1,), (50.0, 40.0)), ("deph_t2", (1,), (50.0, 30.0))]
    assert dv.readout_noise(d, [0], 1) == []
    dm = emulate(2, [("x", (0,), ())] + dv.readout_noise(d, [0], 0))
    _, w = om.measure_z(dm, 0, 0.5)
    assert abs(w[0] - 0.001) <= 1e-16 and abs(w[1] - 0.999) <= 1e-15
