"""ctypes front end of the C oracle core (``dm_oracle.c``).  Test infrastructure.

The shared library is compiled with gcc into ``oracle/liboracle.so`` on first
use (or by ``build_oracle()``), with OpenMP for the outer loops.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile dm_oracle.c with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-std=c11", "-shared", "-fPIC",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build_oracle()
            L = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            L.orc_init_zero.argtypes = [dp, ctypes.c_int]
            L.orc_init_basis.argtypes = [dp, ctypes.c_int, ctypes.c_uint64]
            L.orc_init_product_diag.argtypes = [dp, ctypes.c_int, dp]
            L.orc_apply_matrix.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, dp]
            L.orc_apply_kraus.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, dp]
            L.orc_trace.argtypes = [dp, ctypes.c_int, dp, dp]
            L.orc_probs.argtypes = [dp, ctypes.c_int, dp]
            L.orc_expec_z.argtypes = [dp, ctypes.c_int, dp]
            L.orc_expec_zz.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp]
            L.orc_purity.argtypes = [dp, ctypes.c_int]
            L.orc_purity.restype = ctypes.c_double
            L.orc_expec_pauli.argtypes = [dp, ctypes.c_int, ip, dp, dp]
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class OracleDM:
    """An n-qubit density matrix held as a row-major complex128 (2^n, 2^n) array."""

    def __init__(self, n: int):
        if not 1 <= n <= 16:
            raise ValueError("n must be in [1, 16]")
        self.n = n
        D = 1 << n
        self.R = np.zeros((D, D), dtype=np.complex128)
        lib().orc_init_zero(_dp(self.R), n)

    # -- initial states ------------------------------------------------
    def init_zero(self):
        lib().orc_init_zero(_dp(self.R), self.n)

    def init_basis(self, b: int):
        lib().orc_init_basis(_dp(self.R), self.n, int(b))

    def init_product_diag(self, p0):
        p = np.ascontiguousarray(p0, dtype=np.float64)
        assert p.shape == (self.n,)
        lib().orc_init_product_diag(_dp(self.R), self.n, _dp(p))

    def set(self, rho: np.ndarray):
        self.R[...] = rho

    # -- operations ----------------------------------------------------
    def _targets(self, targets):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        if len(set(t.tolist())) != len(t) or t.min() < 0 or t.max() >= self.n:
            raise ValueError("bad targets %r" % (targets,))
        return t

    def apply_matrix(self, targets, M):
        """rho <- M rho M^dagger with M on ``targets`` (targets[0] = LSB)."""
        t = self._targets(targets)
        k = len(t)
        if k > 6:
            raise ValueError("k > 6")
        M = np.ascontiguousarray(M, dtype=np.complex128)
        assert M.shape == (1 << k, 1 << k)
        lib().orc_apply_matrix(_dp(self.R), self.n, k, _ip(t), _dp(M))

    def apply_kraus(self, targets, Ks):
        """rho <- sum_j K_j rho K_j^dagger."""
        t = self._targets(targets)
        k = len(t)
        if k > 4:
            raise ValueError("k > 4")
        K = np.ascontiguousarray(np.stack([np.asarray(x, dtype=np.complex128) for x in Ks]))
        assert K.shape[1:] == (1 << k, 1 << k)
        lib().orc_apply_kraus(_dp(self.R), self.n, k, _ip(t), K.shape[0], _dp(K))

    # -- read-outs -----------------------------------------------------
    def trace(self) -> complex:
        re = ctypes.c_double()
        im = ctypes.c_double()
        lib().orc_trace(_dp(self.R), self.n, ctypes.byref(re), ctypes.byref(im))
        return complex(re.value, im.value)

    def probs(self) -> np.ndarray:
        out = np.empty(1 << self.n)
        lib().orc_probs(_dp(self.R), self.n, _dp(out))
        return out

    def expec_z(self) -> np.ndarray:
        out = np.empty(self.n)
        lib().orc_expec_z(_dp(self.R), self.n, _dp(out))
        return out

    def expec_zz(self, pairs) -> np.ndarray:
        p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out = np.empty(p.shape[0])
        lib().orc_expec_zz(_dp(self.R), self.n, _ip(p), p.shape[0], _dp(out))
        return out

    def purity(self) -> float:
        return float(lib().orc_purity(_dp(self.R), self.n))

    def expec_pauli(self, codes) -> complex:
        c = np.ascontiguousarray(codes, dtype=np.int32)
        assert c.shape == (self.n,)
        re = ctypes.c_double()
        im = ctypes.c_double()
        lib().orc_expec_pauli(_dp(self.R), self.n, _ip(c), ctypes.byref(re), ctypes.byref(im))
        return complex(re.value, im.value)

    def to_vectorised(self) -> np.ndarray:
        """The same state in the vectorised order amp[r + 2^n c] = rho[r][c]."""
        return np.ascontiguousarray(self.R.T).reshape(-1)
