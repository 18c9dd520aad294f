"""Error parameters from gate fidelities (App. B): the oracle's bisection
(oracle/params.py) pinned to the entanglement fidelity that the
density-matrix oracle computes for the recovered channels, and the library's
closed-form inversion against the oracle."""
import math

import numpy as np
import pytest

from oracle import params as op
from oracle.emulator import emulate


def bell(a, b):
    return [("h", (a,), ()), ("matrix", (a, b), (np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0],
                                                            [0, 1, 0, 0]], dtype=complex),))]


def fe_numeric(nq, p_depol, p_deph):
    """<Phi|(E (x) I)(Phi)|Phi> from the density-matrix oracle."""
    if nq == 1:
        ops = bell(0, 1) + [("depol1", (0,), (p_depol,)), ("deph1", (0,), (p_deph,))]
        ref = bell(0, 1)
        n = 2
    else:
        ops = bell(0, 2) + bell(1, 3) + [("depol2", (0, 1), (p_depol,)), ("deph2", (0, 1), (p_deph,))]
        ref = bell(0, 2) + bell(1, 3)
        n = 4
    return float(np.real(np.trace(emulate(n, ref).R @ emulate(n, ops).R)))


CASES = [(1, 0.999, 0.5), (1, 0.99, 0.0), (1, 0.97, 1.0), (1, 0.9, 0.3), (2, 0.995, 0.5), (2, 0.95, 0.8),
         (2, 0.9, 0.0), (2, 0.99, 1.0)]


@pytest.mark.parametrize("nq,F,x", CASES)
def test_oracle_inversion_reproduces_the_fidelity(nq, F, x):
    p, q = op.severity(F, nq, x)
    assert abs(fe_numeric(nq, p, q) - op.ent_from_avg(F, nq)) <= 1e-12
    d = 2 ** nq
    assert abs((d * fe_numeric(nq, p, q) + 1) / (d + 1) - F) <= 1e-12


@pytest.mark.parametrize("nq,F,x", CASES)
def test_library_matches_oracle(vqd_host, nq, F, x):
    p, q = vqd_host.fidelity_to_errors(nq, F, x)
    pr, qr = op.severity(F, nq, x)
    assert abs(p - pr) <= 1e-12 and abs(q - qr) <= 1e-12
    assert abs(vqd_host.entanglement_fidelity(nq, p, q) - op.ent_fidelity(p, q, nq)) <= 1e-15


def test_end_points_and_errors(vqd_host):
    v = vqd_host
    assert v.fidelity_to_errors(1, 1.0, 0.4) == (0.0, 0.0)
    p, q = v.fidelity_to_errors(1, 0.97, 0.0)           # all dephasing: eps = 1 - F_e
    assert p == 0.0 and abs(q - (1 - op.ent_from_avg(0.97, 1))) <= 1e-15
    p, q = v.fidelity_to_errors(2, 0.97, 1.0)
    assert q == 0.0 and abs(p - (1 - op.ent_from_avg(0.97, 2))) <= 1e-15
    for bad in ((3, 0.99, 0.5), (1, 0.99, -0.1), (1, 0.99, 1.1), (1, 1.01, 0.5), (1, 0.1, 0.5)):
        with pytest.raises(v.VQDError):
            v.fidelity_to_errors(*bad)


def test_angle_scaling(vqd_host):
    for eps, th in ((0.01, math.pi), (0.02, -math.pi / 2), (0.3, 0.0), (0.1, 2.5)):
        assert abs(vqd_host.angle_scaled_error(eps, th) - op.angle_scaled(eps, th)) <= 1e-17
    assert vqd_host.angle_scaled_error(0.01, math.pi) == 0.01
