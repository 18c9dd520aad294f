"""The time-parameterised passive channels of Sec. 3.5 that the benchmark
circuits do not use: Gaussian T2* dephasing (eq. depht2s) and depolarising
T1 decay (eq. depolt1).  Oracle pins by their closed forms; the library's
superoperators against the oracle's Kraus sets."""
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


@pytest.mark.parametrize("kind,params", [("deph_t2s", (0.7, 2.0)), ("depol_t1", (0.7, 2.0)),
                                         ("deph_t2s", (0.0, 1.0)), ("depol_t1", (5.0, 0.5))])
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
