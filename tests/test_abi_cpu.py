"""C-ABI checks that need no GPU: every declared symbol is exported, argument
errors are reported with the documented codes before anything is enqueued,
and the host-side builders agree with the oracle's Kraus maps."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import channels as och

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(vqd_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(vqd_host):
    L = ctypes.CDLL(vqd_host.LIB_PATH)
    names = declared_functions()
    assert len(names) > 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_argument_errors(vqd_host):
    L = vqd_host.lib()
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: every call below fails validation
    h = ctypes.c_void_p()
    assert L.vqd_dm_wrap(None, 3, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.vqd_dm_wrap(fake, 0, 1 << 20, None, ctypes.byref(h)) == -2
    assert L.vqd_dm_wrap(fake, 17, 1 << 40, None, ctypes.byref(h)) == -2
    assert L.vqd_dm_wrap(fake, 3, 16 * 64 - 1, None, ctypes.byref(h)) == -2
    assert b"need" in L.vqd_last_error()
    assert L.vqd_dm_wrap(fake, 3, 16 * 64, None, ctypes.byref(h)) == 0
    U = np.eye(2, dtype=np.complex128).view(np.float64)
    dp = U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.vqd_apply_unitary1(h, 3, dp) == -1           # q outside [0, n)
    assert L.vqd_apply_unitary1(h, -1, dp) == -1
    assert L.vqd_apply_unitary2(h, 1, 1, dp) == -1        # duplicate targets
    assert b"duplicate" in L.vqd_last_error()
    assert L.vqd_apply_unitary1(h, 0, None) == -1
    bad = np.eye(2, dtype=np.complex128)
    bad[0, 1] = np.nan
    assert L.vqd_apply_unitary1(h, 0, bad.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -1
    assert b"non-finite" in L.vqd_last_error()
    t = (ctypes.c_int * 3)(0, 1, 2)
    assert L.vqd_apply_fused(h, 3, t, 1, dp) == -2        # superop block needs k <= 2
    assert L.vqd_apply_fused(h, 5, t, 0, dp) == -2
    assert L.vqd_dm_init_basis(h, 8) == -1
    codes = (ctypes.c_uint8 * 3)(0, 4, 0)
    re_, im_ = ctypes.c_double(), ctypes.c_double()
    assert L.vqd_calc_expec_pauli(h, codes, ctypes.byref(re_), ctypes.byref(im_)) == -1
    assert L.vqd_dm_destroy(None) == 0
    p = ctypes.c_void_p()
    assert L.vqd_prog_create(0, ctypes.byref(p)) == -2
    assert L.vqd_prog_create(4, ctypes.byref(p)) == 0
    tq = (ctypes.c_int * 2)(0, 0)
    assert L.vqd_prog_add_named(p, 9, tq, None) == -1    # CZ on a duplicated qubit
    assert L.vqd_prog_add_named(p, 99, tq, None) == -1
    pr = (ctypes.c_double * 1)(1.5)
    tq1 = (ctypes.c_int * 1)(0)
    assert L.vqd_prog_add_named(p, 13, tq1, pr) == -1    # depolarising p > 1
    assert L.vqd_prog_run(p, h) == -5                     # not compiled
    assert L.vqd_prog_destroy(p) == 0


@pytest.mark.parametrize("kind,params", [
    ("depol1", (0.1,)), ("depol2", (0.2,)), ("deph1", (0.3,)), ("deph2", (0.4,)),
    ("amp", (0.25,)), ("gamp", (0.7, 0.2)), ("bitflip1", (0.1,)), ("bitflip2", (0.3,)),
    ("amp_t1", (0.5, 30.0)), ("deph_t2", (0.5, 20.0)), ("parity_decay", ())])
def test_channel_superops_match_oracle_kraus(vqd_host, kind, params):
    S = vqd_host.kind_superop(kind, params)
    Ks = och.CHANNELS[kind](*params)
    d = Ks[0].shape[0]
    # S[(r',c'),(r,c)] = sum_j K[r'][r] conj(K[c'][c]), local index r + d c
    ref = np.zeros((d * d, d * d), dtype=complex)
    for K in Ks:
        for r2 in range(d):
            for c2 in range(d):
                for r in range(d):
                    for c in range(d):
                        ref[r2 + d * c2, r + d * c] += K[r2, r] * np.conj(K[c2, c])
    assert np.abs(S - ref).max() < 1e-15


@pytest.mark.parametrize("kind,params", [
    ("rx", (0.7,)), ("ry", (1.9,)), ("rz", (2.5,)), ("h", ()), ("x", ()), ("y", ()), ("z", ()),
    ("su2", (0.3, -1.1, 0.4, 2.0)), ("cz", ()), ("cphase", (0.6,)), ("xx", (1.1,)), ("zz", (0.01,)),
    ("rabi", (1.7, 0.9, -0.6, 1.3)), ("rabi", (0.0, 0.3, 0.0, 2.0)), ("rabi", (5.0, -2.2, 3.1, 0.21)),
    ("offres", (1.0, 2.0, 0.7)), ("offres", (0.0, 7.0, 0.11)), ("offres", (0.3, 40.0, 1.9)),
    ("crz", (0.45,)), ("crz", (-2.8,))])
def test_gate_matrices_match_oracle(vqd_host, kind, params):
    U = vqd_host.kind_matrix(kind, params)
    assert np.abs(U - och.gate_matrix(kind, params)).max() < 1e-14
