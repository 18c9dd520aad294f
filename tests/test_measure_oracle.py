"""Pins of the measurement oracle (oracle/measure.py): closed forms, the
Born rule on explicit projectors, idempotence, the non-selective average
against the dephasing channel of the density-matrix oracle, Bell-state
parities, and the sampling rule against the per-draw definition."""
import math

import numpy as np
import pytest

from oracle import measure as ms
from oracle.core import OracleDM
from oracle.emulator import emulate
from oracle.trajectories import draw
from workloads import random_tp_ops


def dm_of(n, ops):
    return emulate(n, ops)


def random_rho(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    rho = A @ A.conj().T
    return rho / np.trace(rho)


def test_plus_state_closed_form():
    for u, m in ((0.0, 0), (0.4999, 0), (0.5, 1), (0.9, 1)):
        dm = dm_of(1, [("h", (0,), ())])
        out, w = ms.measure_z(dm, 0, u)
        assert out == m and abs(w[0] - 0.5) <= 1e-15 and abs(w[1] - 0.5) <= 1e-15
        ref = np.zeros((2, 2))
        ref[m, m] = 1
        assert np.abs(dm.R - ref).max() <= 1e-15


@pytest.mark.parametrize("n,q", [(2, 0), (3, 1), (3, 2), (4, 3)])
def test_born_rule_and_collapse_on_a_mixed_state(n, q):
    rho = random_rho(n, 10 + n + q)
    D = 1 << n
    bit = (np.arange(D) >> q) & 1
    for m in (0, 1):
        dm = OracleDM(n)
        dm.set(rho)
        p = [float(np.real(np.trace(rho[np.ix_(bit == k, bit == k)]))) for k in (0, 1)]
        u = 0.5 * p[0] if m == 0 else p[0] + 0.5 * p[1]
        out, w = ms.measure_z(dm, q, u)
        assert out == m and np.allclose(w, p, atol=1e-15)
        keep = np.outer(bit == m, bit == m)
        assert np.abs(dm.R - np.where(keep, rho, 0) / p[m]).max() <= 1e-14
        assert abs(np.trace(dm.R) - 1) <= 1e-14
        # a second measurement repeats the outcome with certainty
        out2, w2 = ms.measure_z(dm, q, 0.999999)
        assert out2 == m and abs(w2[m] - 1) <= 1e-14


def test_nonselective_average_is_full_dephasing():
    """sum_m w_m rho_m equals deph(1/2) on the qubit (eq. deph1 at p = 1/2)."""
    n, q = 3, 1
    rho = random_rho(n, 5)
    avg = np.zeros_like(rho)
    for m in (0, 1):
        dm = OracleDM(n)
        dm.set(rho)
        ws = ms.measure_z(dm, q, 0.0 if m == 0 else 0.999999)[1]
        avg += ws[m] * dm.R
    ref = OracleDM(n)
    ref.set(rho)
    ref.apply_kraus([q], [math.sqrt(0.5) * np.eye(2), math.sqrt(0.5) * np.diag([1, -1])])
    assert np.abs(avg - ref.R).max() <= 1e-14


def test_parity_of_bell_states():
    """|Phi+> has even parity (outcome "1"), |Psi+> odd (outcome "0") for any u;
    an even-odd mixture splits by its weights."""
    phi = [("h", (0,), ()), ("matrix", (0, 1), (np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0],
                                                            [0, 1, 0, 0]], dtype=complex),))]
    psi = phi + [("x", (1,), ())]
    for u in (0.0, 0.5, 0.999):
        dm = dm_of(2, phi)
        before = dm.R.copy()
        out, w = ms.measure_parity(dm, 0, 1, u)
        assert out == 1 and abs(w[1] - 1) <= 1e-15 and np.abs(dm.R - before).max() <= 1e-15
        dm = dm_of(2, psi)
        out, w = ms.measure_parity(dm, 0, 1, u)
        assert out == 0 and abs(w[0] - 1) <= 1e-15
    mix = OracleDM(2)
    mix.set(np.diag([0.1, 0.2, 0.3, 0.4]).astype(complex))
    out, w = ms.measure_parity(mix, 0, 1, 0.45)
    assert np.allclose(w, [0.5, 0.5]) and out == 0
    assert np.allclose(np.diag(mix.R).real, [0, 0.4, 0.6, 0])


def test_parity_on_separate_qubits_matches_the_projector_definition():
    n = 4
    rho = random_rho(n, 21)
    D = 1 << n
    x = np.arange(D)
    par = ((x >> 3) ^ (x >> 1)) & 1          # qubits 3 and 1
    for m, sel in ((0, par == 1), (1, par == 0)):
        dm = OracleDM(n)
        dm.set(rho)
        p0 = float(np.real(np.diag(rho)[par == 1].sum()))
        out, w = ms.measure_parity(dm, 3, 1, 0.5 * p0 if m == 0 else p0 + 1e-9)
        assert out == m
        assert np.abs(dm.R - np.where(np.outer(sel, sel), rho, 0) / w[m]).max() <= 1e-14


def test_sampling_rule():
    p = np.array([0.1, 0.0, 0.2, 0.3, 0.4, -1e-18])
    U = np.array([0.0, 0.05, 0.15, 0.25, 0.35, 0.55, 0.65, 0.999999])
    got = ms.sample(p, U)
    assert list(got) == [0, 0, 2, 2, 3, 3, 4, 4]   # index 1 (zero) and 5 (negative) never drawn
    ref = [draw([max(0.0, v) for v in p], u) for u in U]
    assert list(got) == ref
    rng = np.random.default_rng(1)
    q = rng.random(64) * (rng.random(64) < 0.7)
    U = rng.random(5000)
    assert np.array_equal(ms.sample(q, U), [draw(list(q), u) for u in U])


def test_shot_frequencies_and_a_stabiliser():
    """2000 shots of a 3-qubit GHZ state: only 000 and 111, about half each,
    and Z0 Z1 = +1 on every shot."""
    ops = [("h", (0,), ()), ("matrix", (0, 1), (np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0],
                                                            [0, 1, 0, 0]], dtype=complex),)),
           ("matrix", (1, 2), (np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0],
                                         [0, 1, 0, 0]], dtype=complex),))]
    dm = dm_of(3, ops)
    shots = ms.sample(dm.probs(), np.random.default_rng(2).random(2000))
    assert set(shots.tolist()) <= {0, 7}
    assert abs((shots == 7).mean() - 0.5) <= 5 * 0.5 / math.sqrt(2000)
    z0z1 = (1 - 2 * (shots & 1)) * (1 - 2 * ((shots >> 1) & 1))
    assert np.all(z0z1 == 1)
