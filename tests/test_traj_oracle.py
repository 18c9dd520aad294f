"""Pins of the trajectory oracle (oracle/trajectories.py) against facts that do
not depend on it: brute-force operators, closed forms, and the density-matrix
oracle (itself pinned in test_oracle_pins.py), which the exact average over
every Kraus branch must reproduce."""
import math

import numpy as np
import pytest

from oracle import channels as ch
from oracle import trajectories as tj
from oracle.emulator import emulate
from tests import _brute as bf
from workloads import c1_line_circuit, random_tp_ops, uniforms


def random_psi(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_apply_matrix_matches_bruteforce(n):
    """Arbitrary (non-unitary) matrices on 1..3 targets in random order."""
    rng = np.random.default_rng(40 + n)
    psi = random_psi(n, n)
    for _ in range(12):
        k = int(rng.integers(1, min(3, n) + 1))
        tg = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        M = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        got = tj.apply_matrix(psi, tg, M)
        ref = bf.embed(n, tg, M) @ psi
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        psi = got / np.linalg.norm(got)


def test_unitary_circuit_is_the_matrix_product():
    """With no channel a trajectory is the ordinary state vector; its <Z_q>
    are those of the full Pauli-Z matrices."""
    n = 4
    ops = [op for op in c1_line_circuit(n=n, n_gates=30, seed=5) if not tj.is_channel(op)]
    assert tj.n_channels(ops) == 0
    psi, drawn = tj.run(n, ops, [])
    assert drawn == []
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = 1
    for kind, tg, params in ops:
        ref = bf.embed(n, tg, ch.gate_matrix(kind, params)) @ ref
    assert np.abs(psi - ref).max() <= 1e-12
    for q in range(n):
        codes = [3 if j == q else 0 for j in range(n)]
        zq = np.vdot(ref, bf.pauli_string(codes) @ ref).real
        assert abs(tj.expec_z(psi)[q] - zq) <= 1e-12


def test_amplitude_damping_closed_form():
    """|1> under amp(p): w = (1-p, p); u below 1-p keeps |1>, above decays to |0>."""
    p = 0.3
    ops = [("x", (0,), ()), ("amp", (0,), (p,))]
    for u, z, j in ((1 - p - 1e-9, -1.0, 0), (1 - p + 1e-9, 1.0, 1), (0.0, -1.0, 0), (0.999999, 1.0, 1)):
        psi, drawn = tj.run(1, ops, [u])
        assert drawn == [j]
        assert abs(tj.expec_z(psi)[0] - z) <= 1e-15
        assert abs(tj.norm2(psi) - 1) <= 1e-15


def test_depolarising_draw_intervals():
    """depol1(p) on |0>: I for u < 1-p, then X, Y, Z in thirds of the rest;
    X and Y flip the qubit, Z only adds a sign."""
    p = 0.3
    op = ("depol1", (0,), (p,))
    edges = [0, 1 - p, 1 - 2 * p / 3, 1 - p / 3, 1]
    for j in range(4):
        u = 0.5 * (edges[j] + edges[j + 1])
        psi, drawn = tj.run(1, [op], [u])
        assert drawn == [j]
        assert abs(tj.expec_z(psi)[0] - (-1.0 if j in (1, 2) else 1.0)) <= 1e-15
    psi, _ = tj.run(1, [op], [edges[2] + 0.5 * p / 3])
    assert abs(psi[1] - 1j) <= 1e-15           # Y|0> = i|1> after renormalisation
    psi, _ = tj.run(1, [("h", (0,), ()), op], [edges[3] + 0.5 * p / 3])
    assert np.abs(psi - np.array([1, -1]) / math.sqrt(2)).max() <= 1e-15   # Z|+> = |->


def test_draw_rule_edges():
    assert tj.draw([0.0, 0.5, 0.5], 0.0) == 1          # zero weight is never drawn
    assert tj.draw([0.5, 0.5, 0.0], 0.999999) == 1
    assert tj.draw([0.25, 0.25, 0.5], 0.5) == 2        # strict: running sum must exceed u W
    assert tj.draw([2.0, 2.0], 0.49) == 0              # weights need not sum to one
    assert tj.draw([1.0, 0.0], 1.0) == 0               # nothing exceeds: last positive weight


def _enumerate(n, ops, psi, prob, i, acc):
    """Every Kraus branch, each taken by the uniform at the middle of its
    interval; accumulates prob * |psi><psi|."""
    if i == len(ops):
        acc += prob * np.outer(psi, psi.conj())
        return
    op = ops[i]
    if not tj.is_channel(op):
        nxt, _, _ = tj.step(psi, op)
        _enumerate(n, ops, nxt, prob, i + 1, acc)
        return
    w = tj.kraus_weights(psi, op[1], ch.build(op)[1])
    W = sum(w)
    cum = 0.0
    for j, x in enumerate(w):
        if x > 0:
            u = (cum + 0.5 * x) / W
            nxt, jj, _ = tj.step(psi, op, u)
            assert jj == j
            _enumerate(n, ops, nxt, prob * x / W, i + 1, acc)
        cum += x


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (2, 3), (3, 4)])
def test_branch_average_is_the_density_matrix(n, seed):
    """The probability-weighted sum over all branches equals the channel
    sequence applied to |0><0| by the density-matrix oracle."""
    ops = random_tp_ops(n, 5, seed=seed, max_k=min(2, n))
    if n >= 2:
        ops = ops + [("amp", (0,), (0.3,)), ("gamp", (n - 1,), (0.4, 0.2)), ("depol2", (0, 1), (0.1,)),
                     ("deph_t2", (1,), (0.5, 2.0))]
    acc = np.zeros((1 << n, 1 << n), dtype=complex)
    _enumerate(n, ops, tj.initial_state(n), 1.0, 0, acc)
    ref = emulate(n, ops).R
    assert np.abs(acc - ref).max() <= 1e-12


def test_mean_converges_to_density_matrix():
    """Sampled trajectories of a noisy 3-qubit line circuit: every <Z_q> lies
    within 5 standard errors of the exact value."""
    n = 3
    ops = c1_line_circuit(n=n, n_gates=12, seed=9)
    ops = [(k, q, (10 * p[0],) if k == "depol1" else p) for k, q, p in ops]   # make the noise visible
    U = uniforms(3000, tj.n_channels(ops), seed=17)
    Z, N = tj.run_many(n, ops, U)
    assert np.abs(N - 1).max() <= 1e-12
    mean, se = tj.estimate(Z)
    exact = emulate(n, ops).expec_z()
    assert np.all(np.abs(mean - exact) <= 5 * se + 1e-12), (mean, exact, se)
    assert se.max() > 0


def test_uniform_count_is_checked():
    ops = [("depol1", (0,), (0.1,)), ("amp", (0,), (0.2,))]
    with pytest.raises(ValueError):
        tj.run(1, ops, [0.5])
    with pytest.raises(ValueError):
        tj.run(1, ops, [0.5, 0.5, 0.5])


def test_estimate_standard_error():
    x = np.array([[1.0], [3.0], [5.0], [7.0]])
    mean, se = tj.estimate(x)
    assert mean[0] == 4.0
    assert abs(se[0] - math.sqrt(20.0 / 3.0) / 2.0) <= 1e-15
