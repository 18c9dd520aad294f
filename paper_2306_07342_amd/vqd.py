"""Thin Python binding of libvqd.so (include/vqd.h).

Only argument marshalling happens here: torch provides the device buffer and
the stream, every step of the emulation runs in the library's HIP kernels.
If the library is not built the binding raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvqd.so")

_lib = None

# op kind names -> enum vqd_kind (include/vqd.h)
KINDS = {
    "rx": 1, "ry": 2, "rz": 3, "h": 4, "x": 5, "y": 6, "z": 7, "su2": 8,
    "cz": 9, "cphase": 10, "xx": 11, "zz": 12,
    "depol1": 13, "depol2": 14, "deph1": 15, "deph2": 16, "amp": 17, "gamp": 18,
    "bitflip1": 19, "bitflip2": 20, "amp_t1": 21, "deph_t2": 22, "deph_t2s": 23, "depol_t1": 24,
    "gamp_t1": 25, "rabi": 26, "offres": 27, "crz": 28, "parity_decay": 29,
}
BLOCK_UNITARY = 0
BLOCK_SUPEROP = 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)


class VQDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("vqd error %d: %s" % (code, msg))
        self.code = code


class PlanOpts(ctypes.Structure):
    _fields_ = [("tile_bits", ctypes.c_int), ("min_contig_bits", ctypes.c_int),
                ("max_ops_per_pass", ctypes.c_int), ("fuse_blocks", ctypes.c_int),
                ("pad_coalesce", ctypes.c_int), ("hermitian", ctypes.c_int), ("relayout", ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int), ("total_passes", ctypes.c_longlong),
                ("arena_bytes", ctypes.c_size_t), ("n_outputs", ctypes.c_size_t),
                ("grid_items", ctypes.c_uint), ("fp64_fma", ctypes.c_double), ("pass_bytes", ctypes.c_double)]


class ProgInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_ops", ctypes.c_int), ("n_passes", ctypes.c_int),
                ("n_phases", ctypes.c_int), ("n_kernel_ops", ctypes.c_int),
                ("fma_per_amp", ctypes.c_double), ("hermitian", ctypes.c_int),
                ("tile_fraction", ctypes.c_double), ("relabelled", ctypes.c_int),
                ("layout_changes", ctypes.c_int)]


class TrajInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_ops", ctypes.c_int), ("n_channels", ctypes.c_int),
                ("n_phases", ctypes.c_int), ("n_kernel_ops", ctypes.c_int), ("n_mixed", ctypes.c_int),
                ("n_general", ctypes.c_int), ("fma_per_amp", ctypes.c_double)]


def load(path: str = LIB_PATH):
    """Load libvqd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libvqd.so is not built (%s); run `python -m paper_2306_07342_amd.build`" % path)
    # PyTorch (which provides device memory and streams) must bring up the GPU
    # before the library's HIP runtime does: loading the library registers
    # its kernels, and a device first opened by that runtime cannot then be
    # initialised by PyTorch's
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    sig = {
        "vqd_last_error": ([], ctypes.c_char_p),
        "vqd_version": ([], ctypes.c_char_p),
        "vqd_dm_wrap": ([vp, ctypes.c_int, ctypes.c_size_t, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "vqd_dm_destroy": ([vp], ctypes.c_int),
        "vqd_dm_set_stream": ([vp, vp], ctypes.c_int),
        "vqd_dm_init_zero": ([vp], ctypes.c_int),
        "vqd_dm_init_basis": ([vp, ctypes.c_uint64], ctypes.c_int),
        "vqd_dm_init_product_diag": ([vp, _dp], ctypes.c_int),
        "vqd_dm_copy_to_host": ([vp, _dp], ctypes.c_int),
        "vqd_dm_copy_from_host": ([vp, _dp], ctypes.c_int),
        "vqd_apply_unitary1": ([vp, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_apply_unitary2": ([vp, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_apply_superop1": ([vp, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_apply_superop2": ([vp, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_apply_fused": ([vp, ctypes.c_int, _ip, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_apply_diagonal": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_kind_arity": ([ctypes.c_int, _ip, _ip], ctypes.c_int),
        "vqd_kind_matrix": ([ctypes.c_int, _dp, _dp], ctypes.c_int),
        "vqd_kind_superop": ([ctypes.c_int, _dp, _dp], ctypes.c_int),
        "vqd_kraus_to_superop": ([ctypes.c_int, ctypes.c_int, _dp, _dp], ctypes.c_int),
        "vqd_prog_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "vqd_prog_destroy": ([vp], ctypes.c_int),
        "vqd_prog_add_named": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_prog_add_unitary": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_prog_add_named_many": ([vp, ctypes.c_int, _ip, _ip, _dp], ctypes.c_int),
        "vqd_prog_add_superop": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_prog_add_kraus": ([vp, ctypes.c_int, _ip, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_plan_opts_default": ([ctypes.POINTER(PlanOpts)], None),
        "vqd_prog_compile": ([vp, ctypes.POINTER(PlanOpts)], ctypes.c_int),
        "vqd_prog_plan": ([vp, ctypes.POINTER(PlanOpts)], ctypes.c_int),
        "vqd_prog_export": ([vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vqd_prog_run": ([vp, vp], ctypes.c_int),
        "vqd_prog_info_get": ([vp, ctypes.POINTER(ProgInfo)], ctypes.c_int),
        "vqd_batch_create": ([ctypes.POINTER(vp)], ctypes.c_int),
        "vqd_batch_destroy": ([vp], ctypes.c_int),
        "vqd_batch_add": ([vp, vp, _ip], ctypes.c_int),
        "vqd_batch_set_opts": ([vp, ctypes.c_int, ctypes.POINTER(PlanOpts)], ctypes.c_int),
        "vqd_batch_plan_opts": ([vp, ctypes.c_int, ctypes.POINTER(PlanOpts)], ctypes.c_int),
        "vqd_batch_compile": ([vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vqd_batch_offsets": ([vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vqd_batch_run": ([vp, vp, ctypes.c_size_t, _dp, vp, ctypes.c_int], ctypes.c_int),
        "vqd_batch_autotune": ([vp, vp, ctypes.c_size_t, _dp, vp, ctypes.c_char_p, ctypes.c_int], ctypes.c_int),
        "vqd_batch_info_get": ([vp, ctypes.POINTER(BatchInfo)], ctypes.c_int),
        "vqd_batch_add_template": ([vp, ctypes.c_int, ctypes.c_int, _ip, _ip, _ip], ctypes.c_int),
        "vqd_batch_add_instances": ([vp, ctypes.c_int, ctypes.c_int, _dp, _ip], ctypes.c_int),
        "vqd_mlp_create": ([ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "vqd_mlp_destroy": ([vp], ctypes.c_int),
        "vqd_mlp_n_params": ([], ctypes.c_int),
        "vqd_mlp_set_state": ([vp, ctypes.c_int, _fp], ctypes.c_int),
        "vqd_mlp_get_state": ([vp, ctypes.c_int, _fp], ctypes.c_int),
        "vqd_mlp_set_step": ([vp, ctypes.c_longlong], ctypes.c_int),
        "vqd_mlp_get_step": ([vp], ctypes.c_longlong),
        "vqd_mlp_grad": ([vp, vp, vp, vp, ctypes.c_int, vp, vp], ctypes.c_int),
        "vqd_mlp_train_step": ([vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, vp, vp], ctypes.c_int),
        "vqd_mlp_predict": ([vp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "vqd_template_export": ([ctypes.c_int, ctypes.c_int, _ip, _ip, _dp, ctypes.POINTER(PlanOpts), vp,
                                 ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vqd_traj_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "vqd_traj_destroy": ([vp], ctypes.c_int),
        "vqd_traj_add_named": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_traj_add_named_many": ([vp, ctypes.c_int, _ip, _ip, _dp], ctypes.c_int),
        "vqd_traj_add_unitary": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_traj_add_kraus": ([vp, ctypes.c_int, _ip, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_traj_plan": ([vp], ctypes.c_int),
        "vqd_traj_export": ([vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "vqd_traj_compile": ([vp], ctypes.c_int),
        "vqd_traj_info_get": ([vp, ctypes.POINTER(TrajInfo)], ctypes.c_int),
        "vqd_traj_run": ([vp, vp, ctypes.c_longlong, vp, vp, vp, vp], ctypes.c_int),
        "vqd_traj_stats": ([vp, ctypes.c_longlong, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "vqd_measure_z": ([vp, ctypes.c_int, ctypes.c_double, _ip, _dp], ctypes.c_int),
        "vqd_measure_parity": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip, _dp], ctypes.c_int),
        "vqd_sample": ([vp, vp, ctypes.c_longlong, vp], ctypes.c_int),
        "vqd_entanglement_fidelity": ([ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp], ctypes.c_int),
        "vqd_fidelity_to_errors": ([ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp], ctypes.c_int),
        "vqd_angle_scaled_error": ([ctypes.c_double, ctypes.c_double], ctypes.c_double),
        "vqd_zz_crosstalk_strength": ([ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp],
                                      ctypes.c_int),
        "vqd_device_create": ([ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "vqd_device_destroy": ([vp], ctypes.c_int),
        "vqd_device_set_gate": ([vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double],
                                ctypes.c_int),
        "vqd_device_set_passive": ([vp, _dp, _dp], ctypes.c_int),
        "vqd_device_set_crosstalk": ([vp, ctypes.c_int, _ip, ctypes.c_double], ctypes.c_int),
        "vqd_device_preset": ([ctypes.c_int, ctypes.POINTER(vp), _dp], ctypes.c_int),
        "vqd_device_preset_qubits": ([ctypes.c_int, _ip], ctypes.c_int),
        "vqd_device_set_gate_on": ([vp, ctypes.c_int, ctypes.c_int, _ip, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double], ctypes.c_int),
        "vqd_device_set_angle_scaling": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "vqd_device_set_thermal": ([vp, _dp], ctypes.c_int),
        "vqd_device_set_passive_forms": ([vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "vqd_device_set_static_zz": ([vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
        "vqd_device_set_readout": ([vp, ctypes.c_double, _dp], ctypes.c_int),
        "vqd_device_set_off_resonant": ([vp, _dp, _dp], ctypes.c_int),
        "vqd_device_set_serial": ([vp, ctypes.c_int], ctypes.c_int),
        "vqd_device_set_readout_form": ([vp, ctypes.c_int], ctypes.c_int),
        "vqd_device_set_parity_readout": ([vp, ctypes.c_double, ctypes.c_double], ctypes.c_int),
        "vqd_device_parity_readout_noise": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip,
                                             _ip, _dp], ctypes.c_int),
        "vqd_device_set_exchange_crosstalk": ([vp, ctypes.c_int, _ip, _dp, _dp], ctypes.c_int),
        "vqd_device_readout_noise": ([vp, ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _ip, _ip, _ip, _dp],
                                     ctypes.c_int),
        "vqd_device_insert_noise": ([vp, ctypes.c_int, _ip, _ip, _dp, ctypes.c_int, _ip, _ip, _ip, _dp],
                                    ctypes.c_int),
        "vqd_calc_trace": ([vp, _dp, _dp], ctypes.c_int),
        "vqd_calc_purity": ([vp, _dp], ctypes.c_int),
        "vqd_calc_probs": ([vp, _dp], ctypes.c_int),
        "vqd_calc_expec_z": ([vp, _dp], ctypes.c_int),
        "vqd_calc_expec_zz": ([vp, _ip, ctypes.c_int, _dp], ctypes.c_int),
        "vqd_calc_expec_pauli": ([vp, ctypes.POINTER(ctypes.c_uint8), _dp, _dp], ctypes.c_int),
        "vqd_calc_trace_dev": ([vp, vp], ctypes.c_int),
        "vqd_calc_purity_dev": ([vp, vp], ctypes.c_int),
        "vqd_calc_probs_dev": ([vp, vp], ctypes.c_int),
        "vqd_calc_expec_z_dev": ([vp, vp], ctypes.c_int),
        "vqd_calc_expec_zz_dev": ([vp, vp, ctypes.c_int, vp], ctypes.c_int),
        "vqd_calc_expec_pauli_dev": ([vp, ctypes.POINTER(ctypes.c_uint8), vp], ctypes.c_int),
        "vqd_calc_expec_z_noalloc": ([vp, ctypes.c_int, vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def lib():
    return _lib if _lib is not None else load()


def check(rc: int):
    if rc != 0:
        raise VQDError(rc, lib().vqd_last_error().decode())


def _cplx(M) -> np.ndarray:
    """Row-major interleaved (re, im) doubles."""
    a = np.ascontiguousarray(np.asarray(M, dtype=np.complex128))
    return a.view(np.float64).reshape(-1)


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _i(a: np.ndarray):
    return a.ctypes.data_as(_ip)


def _stream_ptr(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def kind_superop(kind: str, params: Sequence[float]) -> np.ndarray:
    nq, np_ = ctypes.c_int(), ctypes.c_int()
    check(lib().vqd_kind_arity(KINDS[kind], ctypes.byref(nq), ctypes.byref(np_)))
    d = 4 ** nq.value
    out = np.empty(2 * d * d)
    p = np.ascontiguousarray(params, dtype=np.float64) if len(params) else np.zeros(1)
    check(lib().vqd_kind_superop(KINDS[kind], _d(p), _d(out)))
    return out.view(np.complex128).reshape(d, d)


def kind_matrix(kind: str, params: Sequence[float]) -> np.ndarray:
    nq, np_ = ctypes.c_int(), ctypes.c_int()
    check(lib().vqd_kind_arity(KINDS[kind], ctypes.byref(nq), ctypes.byref(np_)))
    d = 2 ** nq.value
    out = np.empty(2 * d * d)
    p = np.ascontiguousarray(params, dtype=np.float64) if len(params) else np.zeros(1)
    check(lib().vqd_kind_matrix(KINDS[kind], _d(p), _d(out)))
    return out.view(np.complex128).reshape(d, d)


def kraus_to_superop(Ks) -> np.ndarray:
    K = np.ascontiguousarray(np.stack([np.asarray(x, dtype=np.complex128) for x in Ks]))
    d = K.shape[1]
    k = int(round(np.log2(d)))
    out = np.empty(2 * d ** 4)
    check(lib().vqd_kraus_to_superop(k, K.shape[0], _d(_cplx(K)), _d(out)))
    return out.view(np.complex128).reshape(d * d, d * d)


def entanglement_fidelity(nq: int, p_depol: float, p_deph: float) -> float:
    """App. B: entanglement fidelity of depolarising then dephasing noise."""
    out = ctypes.c_double()
    check(lib().vqd_entanglement_fidelity(nq, p_depol, p_deph, ctypes.byref(out)))
    return out.value


def fidelity_to_errors(nq: int, fbar: float, x: float):
    """App. B: (p_depol, p_deph) = (x eps, (1 - x) eps) reproducing average
    gate fidelity fbar."""
    p, q = ctypes.c_double(), ctypes.c_double()
    check(lib().vqd_fidelity_to_errors(nq, fbar, x, ctypes.byref(p), ctypes.byref(q)))
    return p.value, q.value


def angle_scaled_error(eps: float, theta: float) -> float:
    return lib().vqd_angle_scaled_error(eps, theta)


def zz_crosstalk_strength(J: float, delta_ct: float, alpha_c: float, alpha_t: float) -> float:
    """Sec. 8: static ZZ coupling of two transmons (same frequency unit in and out)."""
    out = ctypes.c_double()
    check(lib().vqd_zz_crosstalk_strength(J, delta_ct, alpha_c, alpha_t, ctypes.byref(out)))
    return out.value


class DensityMatrix:
    """An n-qubit density matrix in GPU memory (vectorised, complex128).

    The buffer is a torch float64 tensor of 2 * 4^n values (interleaved
    re, im) with amp[r + 2^n c] = rho[r][c]."""

    def __init__(self, n: int, device="cuda", stream=None, buffer=None):
        import torch
        load()
        self.n = n
        if buffer is None:
            buffer = torch.empty(2 * 4 ** n, dtype=torch.float64, device=device)
        self.buffer = buffer
        h = ctypes.c_void_p()
        check(lib().vqd_dm_wrap(ctypes.c_void_p(buffer.data_ptr()), n,
                                buffer.numel() * buffer.element_size(), _stream_ptr(stream),
                                ctypes.byref(h)))
        self.handle = h
        self.init_zero()

    def close(self):
        if getattr(self, "handle", None):
            check(lib().vqd_dm_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ---------------------------------------------------------
    def init_zero(self):
        check(lib().vqd_dm_init_zero(self.handle))

    def init_basis(self, b: int):
        check(lib().vqd_dm_init_basis(self.handle, int(b)))

    def init_product_diag(self, p0):
        p = np.ascontiguousarray(p0, dtype=np.float64)
        check(lib().vqd_dm_init_product_diag(self.handle, _d(p)))

    def to_numpy(self) -> np.ndarray:
        """Vectorised amplitudes as complex128[4^n] (synchronous copy)."""
        out = np.empty(2 * 4 ** self.n)
        check(lib().vqd_dm_copy_to_host(self.handle, _d(out)))
        return out.view(np.complex128)

    def to_matrix(self) -> np.ndarray:
        """rho as a (2^n, 2^n) matrix (rho[r][c] = amp[r + 2^n c])."""
        D = 1 << self.n
        return self.to_numpy().reshape(D, D).T.copy()

    def from_numpy(self, amps: np.ndarray):
        a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128).reshape(-1))
        check(lib().vqd_dm_copy_from_host(self.handle, _d(a.view(np.float64))))

    # -- ops -----------------------------------------------------------
    def apply_unitary1(self, q, U):
        check(lib().vqd_apply_unitary1(self.handle, int(q), _d(_cplx(U))))

    def apply_unitary2(self, q0, q1, U):
        check(lib().vqd_apply_unitary2(self.handle, int(q0), int(q1), _d(_cplx(U))))

    def apply_superop1(self, q, S):
        check(lib().vqd_apply_superop1(self.handle, int(q), _d(_cplx(S))))

    def apply_superop2(self, q0, q1, S):
        check(lib().vqd_apply_superop2(self.handle, int(q0), int(q1), _d(_cplx(S))))

    def apply_fused(self, targets, M, kind=BLOCK_UNITARY):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        check(lib().vqd_apply_fused(self.handle, len(t), _i(t), kind, _d(_cplx(M))))

    def apply_diagonal(self, targets, d):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        check(lib().vqd_apply_diagonal(self.handle, len(t), _i(t), _d(_cplx(d))))

    # -- read-out ------------------------------------------------------
    def trace(self) -> complex:
        re, im = ctypes.c_double(), ctypes.c_double()
        check(lib().vqd_calc_trace(self.handle, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def purity(self) -> float:
        out = ctypes.c_double()
        check(lib().vqd_calc_purity(self.handle, ctypes.byref(out)))
        return out.value

    def probs(self) -> np.ndarray:
        out = np.empty(1 << self.n)
        check(lib().vqd_calc_probs(self.handle, _d(out)))
        return out

    def expec_z(self) -> np.ndarray:
        out = np.empty(self.n)
        check(lib().vqd_calc_expec_z(self.handle, _d(out)))
        return out

    def expec_zz(self, pairs) -> np.ndarray:
        p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out = np.empty(p.shape[0])
        check(lib().vqd_calc_expec_zz(self.handle, _i(p), p.shape[0], _d(out)))
        return out

    def measure_z(self, q: int, u: float):
        """Projective Z measurement of qubit q with uniform u (vqd_measure_z);
        collapses the state, returns (outcome, weight)."""
        m, w = ctypes.c_int(), ctypes.c_double()
        check(lib().vqd_measure_z(self.handle, q, float(u), ctypes.byref(m), ctypes.byref(w)))
        return m.value, w.value

    def measure_parity(self, q0: int, q1: int, u: float):
        """Parity measurement of eq. (m) (outcome 0 odd, 1 even); collapses the
        state, returns (outcome, weight)."""
        m, w = ctypes.c_int(), ctypes.c_double()
        check(lib().vqd_measure_parity(self.handle, q0, q1, float(u), ctypes.byref(m), ctypes.byref(w)))
        return m.value, w.value

    def sample(self, uniforms, out=None):
        """One basis state per uniform (a CUDA float64 tensor) from the diagonal
        probabilities (vqd_sample); returns a CUDA int32 tensor of bit strings."""
        import torch
        if not (uniforms.is_cuda and uniforms.dtype == torch.float64 and uniforms.is_contiguous()):
            raise ValueError("uniforms must be a contiguous CUDA float64 tensor")
        shots = uniforms.numel()
        if out is None:
            out = torch.empty(shots, dtype=torch.int32, device=uniforms.device)
        check(lib().vqd_sample(self.handle, ctypes.c_void_p(uniforms.data_ptr()), shots,
                               ctypes.c_void_p(out.data_ptr())))
        return out

    def expec_pauli(self, codes) -> complex:
        c = np.ascontiguousarray(codes, dtype=np.uint8)
        re, im = ctypes.c_double(), ctypes.c_double()
        check(lib().vqd_calc_expec_pauli(self.handle, c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                         ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    # -- device-output read-outs (asynchronous, no allocation; capturable) --
    @staticmethod
    def _dev_out(t, count: int, dtype_name: str = "float64"):
        import torch
        want = getattr(torch, dtype_name)
        if not (t.is_cuda and t.dtype == want and t.is_contiguous() and t.numel() >= count):
            raise ValueError("output must be a contiguous CUDA %s tensor of at least %d elements"
                             % (dtype_name, count))
        return ctypes.c_void_p(t.data_ptr())

    def trace_dev(self, out):
        """vqd_calc_trace_dev: (re, im) into out[0:2]."""
        check(lib().vqd_calc_trace_dev(self.handle, self._dev_out(out, 2)))
        return out

    def purity_dev(self, out):
        check(lib().vqd_calc_purity_dev(self.handle, self._dev_out(out, 1)))
        return out

    def probs_dev(self, out):
        check(lib().vqd_calc_probs_dev(self.handle, self._dev_out(out, 1 << self.n)))
        return out

    def expec_z_dev(self, out):
        check(lib().vqd_calc_expec_z_dev(self.handle, self._dev_out(out, self.n)))
        return out

    def expec_zz_dev(self, pairs, out):
        """pairs: CUDA int32 tensor (npairs, 2)."""
        npairs = pairs.numel() // 2
        check(lib().vqd_calc_expec_zz_dev(self.handle, self._dev_out(pairs, 2 * npairs, "int32"), npairs,
                                          self._dev_out(out, npairs)))
        return out

    def expec_pauli_dev(self, codes, out):
        c = np.ascontiguousarray(codes, dtype=np.uint8)
        check(lib().vqd_calc_expec_pauli_dev(self.handle, c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                             self._dev_out(out, 2)))
        return out


def calc_expec_z_noalloc(amps, n: int, out, stream=None):
    """vqd_calc_expec_z_noalloc: <Z_i> of the state in the CUDA float64 tensor
    `amps` (2 * 4^n values) into the CUDA float64 tensor `out` (n values),
    without a handle and without any allocation by the library."""
    for t, count in ((amps, 2 * 4 ** n), (out, n)):
        if not (t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float64" and t.numel() >= count):
            raise ValueError("amps and out must be contiguous CUDA float64 tensors of 2*4^n and n values")
    check(lib().vqd_calc_expec_z_noalloc(ctypes.c_void_p(amps.data_ptr()), n, _stream_ptr(stream),
                                         ctypes.c_void_p(out.data_ptr())))
    return out


def plan_opts(tile_bits=13, min_contig_bits=3, max_ops_per_pass=0, fuse_blocks=True,
              pad_coalesce=True, hermitian=False, relayout=False) -> PlanOpts:
    return PlanOpts(tile_bits, min_contig_bits, max_ops_per_pass, 1 if fuse_blocks else 0,
                    1 if pad_coalesce else 0, 1 if hermitian else 0, 1 if relayout else 0)


def _structure(structure):
    """(kind, qubits) pairs -> int32 kind codes and an (n_ops, 4) target array."""
    k = np.fromiter((KINDS[s[0]] for s in structure), dtype=np.int32)
    t = np.zeros((len(k), 4), dtype=np.int32)
    for i, s in enumerate(structure):
        t[i, :len(s[1])] = s[1]
    return k, t


def template_export(n: int, structure, params=None, opts: Optional[PlanOpts] = None) -> bytes:
    """Host-only plan of a parametric template (see vqd_template_export),
    with the coefficients of `params` ((n_ops, 4) array) or the generic ones."""
    k, t = _structure(structure)
    p = None
    if params is not None:
        p = np.ascontiguousarray(params, dtype=np.float64)
        assert p.shape == (len(k), 4), p.shape
    L = lib()
    need = ctypes.c_size_t()
    o = ctypes.byref(opts) if opts is not None else None
    check(L.vqd_template_export(n, len(k), _i(k), _i(t), _d(p) if p is not None else None, o, None, 0,
                                ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    check(L.vqd_template_export(n, len(k), _i(k), _i(t), _d(p) if p is not None else None, o, buf,
                                need.value, ctypes.byref(need)))
    return buf.raw


class Program:
    """An op program planned by the library into fused HBM passes."""

    def __init__(self, n: int, ops: Optional[Iterable] = None):
        load()
        self.n = n
        h = ctypes.c_void_p()
        check(lib().vqd_prog_create(n, ctypes.byref(h)))
        self.handle = h
        if ops is not None:
            self.extend(ops)

    def close(self):
        if getattr(self, "handle", None):
            check(lib().vqd_prog_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, op):
        kind, qubits, params = op
        t = np.ascontiguousarray(qubits, dtype=np.int32)
        if kind == "matrix":
            check(lib().vqd_prog_add_unitary(self.handle, len(t), _i(t), _d(_cplx(params[0]))))
        elif kind == "kraus":
            K = np.stack([np.asarray(x, dtype=np.complex128) for x in params])
            check(lib().vqd_prog_add_kraus(self.handle, len(t), _i(t), K.shape[0], _d(_cplx(K))))
        elif kind == "superop":
            check(lib().vqd_prog_add_superop(self.handle, len(t), _i(t), _d(_cplx(params[0]))))
        else:
            p = np.ascontiguousarray(params, dtype=np.float64) if len(params) else np.zeros(1)
            check(lib().vqd_prog_add_named(self.handle, KINDS[kind], _i(t), _d(p)))

    def extend(self, ops: Iterable):
        """Append ops; runs of named ops are passed in one call."""
        run = []

        def flush():
            if not run:
                return
            k = np.fromiter((KINDS[o[0]] for o in run), dtype=np.int32, count=len(run))
            t = np.zeros((len(run), 4), dtype=np.int32)
            pr = np.zeros((len(run), 4), dtype=np.float64)
            for i, (_, q, par) in enumerate(run):
                t[i, :len(q)] = q
                pr[i, :len(par)] = par
            check(lib().vqd_prog_add_named_many(self.handle, len(run), _i(k), _i(t), _d(pr)))
            run.clear()

        for op in ops:
            if op[0] in KINDS:
                run.append(op)
            else:
                flush()
                self.add(op)
        flush()

    def compile(self, opts: Optional[PlanOpts] = None):
        check(lib().vqd_prog_compile(self.handle, ctypes.byref(opts) if opts is not None else None))
        return self

    def plan(self, opts: Optional[PlanOpts] = None):
        """Plan on the host only (no device needed)."""
        check(lib().vqd_prog_plan(self.handle, ctypes.byref(opts) if opts is not None else None))
        return self

    def export(self) -> bytes:
        """Planned descriptors (see vqd_prog_export in include/vqd.h)."""
        need = ctypes.c_size_t()
        check(lib().vqd_prog_export(self.handle, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        check(lib().vqd_prog_export(self.handle, buf, need.value, ctypes.byref(need)))
        return buf.raw

    def run(self, dm: DensityMatrix):
        check(lib().vqd_prog_run(self.handle, dm.handle))

    def info(self) -> dict:
        i = ProgInfo()
        check(lib().vqd_prog_info_get(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in ProgInfo._fields_}


KIND_NAMES = {v: k for k, v in KINDS.items()}


PRESETS = {"superconducting": 1, "trapped_ion": 2, "silicon": 3}


class Device:
    """Virtual-device noise insertion (vqd_device_* in include/vqd.h): ideal
    gates in, the device's noisy op stream out (host only)."""

    def __init__(self, n: int):
        load()
        self.n = n
        h = ctypes.c_void_p()
        check(lib().vqd_device_create(n, ctypes.byref(h)))
        self.handle = h

    @classmethod
    def preset(cls, name: str):
        """(device, p0): a device of the paper's parameter tables and the
        ground populations of its initial state."""
        load()
        n = ctypes.c_int()
        check(lib().vqd_device_preset_qubits(PRESETS[name], ctypes.byref(n)))
        p0 = np.zeros(n.value)
        h = ctypes.c_void_p()
        check(lib().vqd_device_preset(PRESETS[name], ctypes.byref(h), _d(p0)))
        d = cls.__new__(cls)
        d.n, d.handle = n.value, h
        return d, p0

    def close(self):
        if getattr(self, "handle", None):
            check(lib().vqd_device_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_gate(self, kind: str, duration: float, p_depol: float = 0.0, p_deph: float = 0.0):
        check(lib().vqd_device_set_gate(self.handle, KINDS[kind], duration, p_depol, p_deph))

    def set_passive(self, T1, T2):
        a = np.ascontiguousarray(T1, dtype=np.float64)
        b = np.ascontiguousarray(T2, dtype=np.float64)
        if a.shape != (self.n,) or b.shape != (self.n,):
            raise ValueError("T1 and T2 need one value per qubit")
        check(lib().vqd_device_set_passive(self.handle, _d(a), _d(b)))

    def set_crosstalk(self, edges, alpha: float):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        check(lib().vqd_device_set_crosstalk(self.handle, e.shape[0], _i(e), alpha))

    def set_gate_on(self, kind: str, qubits, duration: float, p_depol: float = 0.0, p_deph: float = 0.0):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        check(lib().vqd_device_set_gate_on(self.handle, KINDS[kind], q.size, _i(q), duration, p_depol, p_deph))

    def set_angle_scaling(self, kind: str, noise: bool = True, duration: bool = False):
        check(lib().vqd_device_set_angle_scaling(self.handle, KINDS[kind], int(noise), int(duration)))

    def _per_qubit(self, v, what):
        a = np.ascontiguousarray(v, dtype=np.float64)
        if a.shape != (self.n,):
            raise ValueError("%s needs one value per qubit" % what)
        return a

    def set_thermal(self, p0):
        a = self._per_qubit(p0, "p0")
        check(lib().vqd_device_set_thermal(self.handle, _d(a)))

    def set_passive_forms(self, t1: str = "amp_t1", t2: str = "deph_t2"):
        check(lib().vqd_device_set_passive_forms(self.handle, KINDS[t1], KINDS[t2]))

    def set_static_zz(self, edges, beta):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        b = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
        if b.shape[0] != e.shape[0]:
            raise ValueError("one coupling per edge")
        check(lib().vqd_device_set_static_zz(self.handle, e.shape[0], _i(e), _d(b) if b.size else None))

    def set_off_resonant(self, rabi=None, freq=None):
        """Off-resonant driving: per-qubit angular Rabi and qubit frequencies;
        rabi None turns it off."""
        if rabi is None:
            check(lib().vqd_device_set_off_resonant(self.handle, None, None))
            return
        r = self._per_qubit(rabi, "rabi")
        f = self._per_qubit(freq, "freq")
        check(lib().vqd_device_set_off_resonant(self.handle, _d(r), _d(f)))

    def set_readout_form(self, kind: str = "depol1"):
        check(lib().vqd_device_set_readout_form(self.handle, KINDS[kind]))

    def set_serial(self, serial: bool = True):
        check(lib().vqd_device_set_serial(self.handle, int(bool(serial))))

    def set_exchange_crosstalk(self, edges, on, off):
        """Residual exchange on `edges`: `on` (one row per active edge) while
        a two-qubit gate runs, `off` otherwise."""
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        m = e.shape[0]
        a = np.ascontiguousarray(on, dtype=np.float64).reshape(-1)
        b = np.ascontiguousarray(off, dtype=np.float64).reshape(-1)
        if a.size != m * m or b.size != m:
            raise ValueError("on needs n_edges^2 values and off n_edges")
        check(lib().vqd_device_set_exchange_crosstalk(self.handle, m, _i(e) if m else None,
                                                      _d(a) if m else None, _d(b) if m else None))

    def set_readout(self, t_meas: float, eps):
        a = self._per_qubit(eps, "eps")
        check(lib().vqd_device_set_readout(self.handle, t_meas, _d(a)))

    @staticmethod
    def _decode(fill) -> list:
        cnt = ctypes.c_int()
        check(fill(0, ctypes.byref(cnt), None, None, None))
        c = cnt.value
        ok = np.zeros(max(c, 1), dtype=np.int32)
        ot = np.zeros((max(c, 1), 4), dtype=np.int32)
        opr = np.zeros((max(c, 1), 4), dtype=np.float64)
        check(fill(c, ctypes.byref(cnt), _i(ok), _i(ot), _d(opr)))
        out = []
        for i in range(c):
            name = KIND_NAMES[int(ok[i])]
            nq, npar = ctypes.c_int(), ctypes.c_int()
            lib().vqd_kind_arity(int(ok[i]), ctypes.byref(nq), ctypes.byref(npar))
            out.append((name, tuple(int(x) for x in ot[i, :nq.value]), tuple(float(x) for x in opr[i, :npar.value])))
        return out

    def insert_noise(self, gates) -> list:
        """Noisy op stream (kind, qubits, params) for a list of named gates."""
        m = len(gates)
        k = np.zeros(max(m, 1), dtype=np.int32)
        t = np.zeros((max(m, 1), 4), dtype=np.int32)
        p = np.zeros((max(m, 1), 4), dtype=np.float64)
        for i, (kind, q, par) in enumerate(gates):
            k[i] = KINDS[kind]
            t[i, :len(q)] = q
            p[i, :len(par)] = par
        return self._decode(lambda cap, cnt, a, b, c: lib().vqd_device_insert_noise(
            self.handle, m, _i(k), _i(t), _d(p), cap, cnt, a, b, c))

    def set_parity_readout(self, t_meas: float, b: float):
        check(lib().vqd_device_set_parity_readout(self.handle, t_meas, b))

    def parity_readout_noise(self, q0: int, q1: int, stage: int) -> list:
        """Noise ops of the parity read-out of (q0, q1): stage 0 before the
        parity projection (ending with the decay map), stage 1 after it."""
        return self._decode(lambda cap, cnt, a, b, c: lib().vqd_device_parity_readout_noise(
            self.handle, q0, q1, stage, cap, cnt, a, b, c))

    def readout_noise(self, qubits, stage: int) -> list:
        """Read-out noise ops of the measured ``qubits``: stage 0 before the
        projective measurement, stage 1 after it."""
        q = np.ascontiguousarray(list(qubits) or [0], dtype=np.int32)
        nq = len(qubits)
        return self._decode(lambda cap, cnt, a, b, c: lib().vqd_device_readout_noise(
            self.handle, nq, _i(q), stage, cap, cnt, a, b, c))


class Trajectories:
    """Monte Carlo state-vector trajectories (vqd_traj_* in include/vqd.h):
    one Kraus operator drawn per channel and trajectory from caller-supplied
    uniforms, the whole state held on the chip."""

    def __init__(self, n: int, ops: Optional[Iterable] = None):
        load()
        self.n = n
        h = ctypes.c_void_p()
        check(lib().vqd_traj_create(n, ctypes.byref(h)))
        self.handle = h
        if ops is not None:
            self.extend(ops)

    def close(self):
        if getattr(self, "handle", None):
            check(lib().vqd_traj_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, op):
        kind, qubits, params = op
        t = np.ascontiguousarray(qubits, dtype=np.int32)
        if kind == "matrix":
            check(lib().vqd_traj_add_unitary(self.handle, len(t), _i(t), _d(_cplx(params[0]))))
        elif kind == "kraus":
            K = np.stack([np.asarray(x, dtype=np.complex128) for x in params])
            check(lib().vqd_traj_add_kraus(self.handle, len(t), _i(t), K.shape[0], _d(_cplx(K))))
        else:
            p = np.ascontiguousarray(params, dtype=np.float64) if len(params) else np.zeros(1)
            check(lib().vqd_traj_add_named(self.handle, KINDS[kind], _i(t), _d(p)))

    def extend(self, ops: Iterable):
        """Append ops; runs of named ops are passed in one call."""
        run = []

        def flush():
            if not run:
                return
            k = np.fromiter((KINDS[o[0]] for o in run), dtype=np.int32, count=len(run))
            t = np.zeros((len(run), 4), dtype=np.int32)
            pr = np.zeros((len(run), 4), dtype=np.float64)
            for i, (_, q, par) in enumerate(run):
                t[i, :len(q)] = q
                pr[i, :len(par)] = par
            check(lib().vqd_traj_add_named_many(self.handle, len(run), _i(k), _i(t), _d(pr)))
            run.clear()

        for op in ops:
            if op[0] in KINDS:
                run.append(op)
            else:
                flush()
                self.add(op)
        flush()
        return self

    def plan(self):
        """Plan on the host only (no device needed)."""
        check(lib().vqd_traj_plan(self.handle))
        return self

    def export(self) -> bytes:
        need = ctypes.c_size_t()
        check(lib().vqd_traj_export(self.handle, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        check(lib().vqd_traj_export(self.handle, buf, need.value, ctypes.byref(need)))
        return buf.raw

    def compile(self):
        check(lib().vqd_traj_compile(self.handle))
        return self

    def info(self) -> dict:
        i = TrajInfo()
        check(lib().vqd_traj_info_get(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in TrajInfo._fields_}

    def run(self, uniforms, count: Optional[int] = None, z_out=None, norm: bool = True, state: bool = False,
            stream=None) -> dict:
        """Run trajectories for the rows of ``uniforms`` (a CUDA float64 tensor
        [count, n_channels]); returns CUDA tensors z [count, n] and, when
        asked for, norm [count] and state [count, 2^n] (complex128)."""
        import torch
        nch = self.info()["n_channels"]
        if count is None:
            count = int(uniforms.shape[0]) if uniforms is not None else 0
        if nch:
            if (uniforms is None or not uniforms.is_cuda or uniforms.dtype != torch.float64
                    or not uniforms.is_contiguous() or uniforms.numel() != count * nch):
                raise ValueError("uniforms must be a contiguous CUDA float64 tensor [count, %d]" % nch)
        dev = uniforms.device if uniforms is not None else torch.device("cuda")
        z = z_out if z_out is not None else torch.empty((count, self.n), dtype=torch.float64, device=dev)
        nrm = torch.empty(count, dtype=torch.float64, device=dev) if norm else None
        st = torch.empty((count, 1 << self.n), dtype=torch.complex128, device=dev) if state else None
        ptr = (lambda x: ctypes.c_void_p(x.data_ptr()) if x is not None else None)
        check(lib().vqd_traj_run(self.handle, ptr(uniforms) if nch else None, count, ptr(z), ptr(nrm), ptr(st),
                                 _stream_ptr(stream)))
        out = {"z": z}
        if norm:
            out["norm"] = nrm
        if state:
            out["state"] = st
        return out

    @staticmethod
    def stats(x, stream=None):
        """Mean over the rows of a CUDA float64 tensor [count, m] and its
        standard error (vqd_traj_stats)."""
        import torch
        x = x.contiguous()
        m = int(x.shape[1]) if x.dim() == 2 else 1
        mean = torch.empty(m, dtype=torch.float64, device=x.device)
        sem = torch.empty(m, dtype=torch.float64, device=x.device)
        check(lib().vqd_traj_stats(ctypes.c_void_p(x.data_ptr()), int(x.shape[0]), m,
                                   ctypes.c_void_p(mean.data_ptr()), ctypes.c_void_p(sem.data_ptr()),
                                   _stream_ptr(stream)))
        return mean, sem


class Batch:
    """Many independent density matrices run by one persistent launch.

    Build with add(n, ops) per instance, then compile(); run() writes <Z_i> of
    every instance into a device float64 tensor and keeps the final states in
    a device arena (both torch-owned)."""

    def __init__(self):
        load()
        h = ctypes.c_void_p()
        check(lib().vqd_batch_create(ctypes.byref(h)))
        self.handle = h
        self.ns = []
        self.arena = None
        self.out = None

    def close(self):
        if getattr(self, "handle", None):
            check(lib().vqd_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, n: int, ops) -> int:
        p = Program(n, ops)
        idx = ctypes.c_int()
        check(lib().vqd_batch_add(self.handle, p.handle, ctypes.byref(idx)))
        p.close()
        self.ns.append(n)
        return idx.value

    def add_template(self, n: int, structure) -> int:
        """A parametric circuit: `structure` is a list of (kind, qubits) named
        ops; instances supply only parameters (add_instances)."""
        k, t = _structure(structure)
        tid = ctypes.c_int()
        check(lib().vqd_batch_add_template(self.handle, n, len(k), _i(k), _i(t), ctypes.byref(tid)))
        self._tmpl = getattr(self, "_tmpl", {})
        self._tmpl[tid.value] = (n, len(k))
        return tid.value

    def add_instances(self, template_id: int, params) -> range:
        """Instances of a template; params has shape (count, n_ops, 4).
        Returns their instance indices."""
        n, n_ops = self._tmpl[template_id]
        p = np.ascontiguousarray(params, dtype=np.float64)
        assert p.ndim == 3 and p.shape[1:] == (n_ops, 4), p.shape
        first = ctypes.c_int()
        check(lib().vqd_batch_add_instances(self.handle, template_id, p.shape[0], _d(p), ctypes.byref(first)))
        self.ns.extend([n] * p.shape[0])
        return range(first.value, first.value + p.shape[0])

    def set_opts(self, n: int, opts: PlanOpts):
        check(lib().vqd_batch_set_opts(self.handle, n, ctypes.byref(opts)))

    def plan_opts(self, n: int) -> dict:
        o = PlanOpts()
        check(lib().vqd_batch_plan_opts(self.handle, n, ctypes.byref(o)))
        return {f: getattr(o, f) for f, _ in PlanOpts._fields_}

    def compile(self, device="cuda"):
        """Plan and upload; (re)allocate the arena and output tensors."""
        import torch
        ab, no = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().vqd_batch_compile(self.handle, ctypes.byref(ab), ctypes.byref(no)))
        need_a = (ab.value + 7) // 8
        if self.arena is None or self.arena.numel() < need_a:
            self.arena = torch.empty(max(need_a, 1), dtype=torch.float64, device=device)
        if self.out is None or self.out.numel() < no.value:
            self.out = torch.empty(max(no.value, 1), dtype=torch.float64, device=device)
        return self

    def ensure_buffers(self, arena_bytes: int, n_outputs: int, device="cuda"):
        import torch
        need_a = (arena_bytes + 7) // 8
        if self.arena is None or self.arena.numel() < need_a:
            self.arena = torch.empty(max(need_a, 1), dtype=torch.float64, device=device)
        if self.out is None or self.out.numel() < n_outputs:
            self.out = torch.empty(max(n_outputs, 1), dtype=torch.float64, device=device)

    def autotune(self, cache_path: str, max_per_n: int = 32, stream=None):
        check(lib().vqd_batch_autotune(self.handle, ctypes.c_void_p(self.arena.data_ptr()),
                                       self.arena.numel() * 8,
                                       ctypes.cast(ctypes.c_void_p(self.out.data_ptr()), _dp),
                                       _stream_ptr(stream), cache_path.encode(), max_per_n))

    def run(self, use_graph: bool = False, stream=None):
        check(lib().vqd_batch_run(self.handle, ctypes.c_void_p(self.arena.data_ptr()),
                                  self.arena.numel() * 8,
                                  ctypes.cast(ctypes.c_void_p(self.out.data_ptr()), _dp),
                                  _stream_ptr(stream), 1 if use_graph else 0))

    def offsets(self, index: int):
        a, o = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().vqd_batch_offsets(self.handle, index, ctypes.byref(a), ctypes.byref(o)))
        return a.value, o.value

    def expec_z(self, index: int):
        """<Z_i> of instance `index` (host copy)."""
        _, o = self.offsets(index)
        return self.out[o:o + self.ns[index]].cpu().numpy()

    def state(self, index: int) -> np.ndarray:
        """Final vectorised state of instance `index` (host copy)."""
        a, _ = self.offsets(index)
        n = self.ns[index]
        v = self.arena[a // 8: a // 8 + 2 * 4 ** n].cpu().numpy()
        return v.view(np.complex128)

    def info(self) -> dict:
        i = BatchInfo()
        check(lib().vqd_batch_info_get(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in BatchInfo._fields_}


class Surrogate:
    """Ensemble of MLPs (24 -> 256 -> 256 -> 256 -> 10, GELU) trained and run
    by the library's bf16/FP32 kernels (see vqd_mlp_* in include/vqd.h).
    Inputs and targets are device float32 tensors."""

    PARAMS, ADAM_M, ADAM_V, GRAD = 0, 1, 2, 3

    def __init__(self, members: int = 4, max_batch: int = 4096, params=None):
        load()
        h = ctypes.c_void_p()
        check(lib().vqd_mlp_create(members, max_batch, ctypes.byref(h)))
        self.handle = h
        self.members = members
        self.max_batch = max_batch
        self.n_params = lib().vqd_mlp_n_params()
        if params is not None:
            self.set_state(self.PARAMS, params)

    def close(self):
        if getattr(self, "handle", None):
            check(lib().vqd_mlp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, which: int, values):
        v = np.ascontiguousarray(values, dtype=np.float32).reshape(self.members, self.n_params)
        check(lib().vqd_mlp_set_state(self.handle, which, v.ctypes.data_as(_fp)))

    def get_state(self, which: int) -> np.ndarray:
        v = np.empty((self.members, self.n_params), dtype=np.float32)
        check(lib().vqd_mlp_get_state(self.handle, which, v.ctypes.data_as(_fp)))
        return v

    @property
    def step(self) -> int:
        return lib().vqd_mlp_get_step(self.handle)

    @step.setter
    def step(self, t: int):
        check(lib().vqd_mlp_set_step(self.handle, int(t)))

    @staticmethod
    def _ptr(t, dtype=None):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    def grad(self, x, y, idx=None, B=None, loss=None, stream=None):
        B = x.shape[0] if B is None and idx is None else (idx.shape[0] if B is None else B)
        check(lib().vqd_mlp_grad(self.handle, self._ptr(x), self._ptr(y), self._ptr(idx), B, self._ptr(loss),
                                 _stream_ptr(stream)))

    def train_step(self, x, y, lr: float, idx=None, B=None, loss=None, stream=None):
        B = x.shape[0] if B is None and idx is None else (idx.shape[0] if B is None else B)
        check(lib().vqd_mlp_train_step(self.handle, self._ptr(x), self._ptr(y), self._ptr(idx), B, float(lr),
                                       self._ptr(loss), _stream_ptr(stream)))

    def predict(self, x, mean=None, spread=None, member_out=None, stream=None):
        """Ensemble mean [B, 10] and spread [B] (device tensors)."""
        import torch
        B = x.shape[0]
        if mean is None:
            mean = torch.empty((B, 10), dtype=torch.float32, device=x.device)
        if spread is None:
            spread = torch.empty(B, dtype=torch.float32, device=x.device)
        check(lib().vqd_mlp_predict(self.handle, self._ptr(x), B, self._ptr(mean), self._ptr(spread),
                                    self._ptr(member_out), _stream_ptr(stream)))
        return mean, spread
