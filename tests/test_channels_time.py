"""The time-parameterised passive channels of Sec. 3.5 that the benchmark
circuits do not use: Gaussian T2* dephasing (eq. depht2s), depolarising T1
decay (eq. depolt1) and T1 relaxation towards a thermal state (eq. gdamp with
gamma(dt) = 1 - exp(-dt/T1), Sec. 8).  Oracle pins by their closed forms; the
library's superoperators against the oracle's Kraus sets."""
import math

import numpy as np
import pytest

from oracle import channels as ch
from oracle.emulator import emulate
from tests import _brute as bf


@pytest.mark.parametrize("t,T", [(0.0, 5.0), (1.0, 5.0), (4.0, 3.0), (20.0, 2.0)])
def test_gaussian_t2star_coherence(t, T):
    """<X> of |+> after deph_t2s(t, T2*) is exp(-(t/T2*)^2)."""
    dm = emulate(1, [("h", (0,), ()), ("deph_t2s", (0,), (t, T))])
    assert abs(dm.expec_pauli([1]).real - math.exp(-(t / T) ** 2)) <= 1e-14


@pytest.mark.parametrize("t,T", [(0.0, 5.0), (1.0, 5.0), (7.0, 3.0), (200.0, 2.0)])
def test_depolarising_t1_population(t, T):
    """<Z> of |0> after depol_t1(t, T1) is exp(-t/T1); the state tends to I/2."""
    dm = emulate(1, [("depol_t1", (0,), (t, T))])
    assert abs(dm.expec_z()[0] - math.exp(-t / T)) <= 1e-14
    assert abs(dm.purity() - 0.5 * (1 + math.exp(-2 * t / T))) <= 1e-14


@pytest.mark.parametrize("p,t,T", [(0.97, 0.0, 5.0), (0.97, 1.0, 5.0), (0.6, 7.0, 3.0), (0.9, 300.0, 2.0)])
@pytest.mark.parametrize("start", ["0", "1", "+"])
def test_thermal_relaxation(p, t, T, start):
    """gamp_t1(p, t, T1): the ground population relaxes exponentially to the
    thermal value, P0(t) = p + (P0(0) - p) e^{-t/T1}, and the coherence
    decays as e^{-t/(2 T1)}; at long times the state is the thermal state of
    eq. thermalstate."""
    prep = {"0": [], "1": [("x", (0,), ())], "+": [("h", (0,), ())]}[start]
    dm = emulate(1, prep + [("gamp_t1", (0,), (p, t, T))])
    P00 = {"0": 1.0, "1": 0.0, "+": 0.5}[start]
    c0 = {"0": 0.0, "1": 0.0, "+": 0.5}[start]
    assert abs(dm.R[0, 0].real - (p + (P00 - p) * math.exp(-t / T))) <= 1e-14
    assert abs(dm.R[0, 1] - c0 * math.exp(-t / (2 * T))) <= 1e-14
    assert abs(np.trace(dm.R) - 1) <= 1e-14


def test_thermal_relaxation_composes_in_time():
    """Relaxing for t1 and then t2 is relaxing for t1 + t2 (the decay is a
    one-parameter semigroup); at p = 1 it is amp_t1."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    rho = A @ A.conj().T
    rho /= np.trace(rho)

    def run(ops):
        from oracle.core import OracleDM
        dm = OracleDM(1)
        dm.set(rho)
        return emulate(1, ops, dm).R

    a = run([("gamp_t1", (0,), (0.8, 0.4, 2.0)), ("gamp_t1", (0,), (0.8, 1.1, 2.0))])
    b = run([("gamp_t1", (0,), (0.8, 1.5, 2.0))])
    assert np.abs(a - b).max() <= 1e-15
    c = run([("gamp_t1", (0,), (1.0, 0.9, 2.0))])
    d = run([("amp_t1", (0,), (0.9, 2.0))])
    assert np.abs(c - d).max() <= 1e-15


@pytest.mark.parametrize("kind,params", [("deph_t2s", (0.7, 2.0)), ("depol_t1", (0.7, 2.0)),
                                         ("deph_t2s", (0.0, 1.0)), ("depol_t1", (5.0, 0.5)),
                                         ("gamp_t1", (0.9, 0.7, 2.0)), ("gamp_t1", (0.0, 5.0, 0.5))])
def test_library_superoperators(vqd_host, kind, params):
    S = vqd_host.kind_superop(kind, params)
    Ks = ch.CHANNELS[kind](*params)
    ref = sum(np.kron(np.conj(K), K) for K in Ks)
    assert np.abs(S - ref).max() <= 1e-15


def test_bad_times(vqd_host):
    for kind in ("deph_t2s", "depol_t1"):
        with pytest.raises(vqd_host.VQDError):
            vqd_host.kind_superop(kind, (1.0, 0.0))
        with pytest.raises(vqd_host.VQDError):
            vqd_host.kind_superop(kind, (-1.0, 2.0))
    for bad in ((0.9, 1.0, 0.0), (0.9, -1.0, 2.0), (1.5, 1.0, 2.0)):
        with pytest.raises(vqd_host.VQDError):
            vqd_host.kind_superop("gamp_t1", bad)
