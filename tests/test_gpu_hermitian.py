"""Hermitian mode of the pass kernel (vqd_plan_opts.hermitian) on the GPU
against the oracle: Hermitian start states, every tile pair (i <= j)
computed once, each off-diagonal tile's conjugate transpose written to its
mirror."""
import sys

import numpy as np
import pytest

from oracle.core import OracleDM
from oracle.emulator import emulate
from workloads import c1_line_circuit, c2_grid_circuit, c3_all_to_all_circuit

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def hermitian_state(n, seed):
    rng = np.random.default_rng(seed)
    D = 1 << n
    A = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    R = A @ A.conj().T
    return R / np.trace(R)


def check(gpu_lib, n, ops, seed, **opts):
    R0 = hermitian_state(n, seed)
    ref = OracleDM(n)
    ref.set(R0)
    emulate(n, ops, ref)
    dm = gpu_lib.DensityMatrix(n)
    dm.from_numpy(np.ascontiguousarray(R0.T).reshape(-1))
    prog = gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(hermitian=True, **opts))
    info = prog.info()
    say("hermitian n=%d ops=%d passes=%d fraction=%.4f" % (n, len(ops), info["n_passes"], info["tile_fraction"]))
    assert info["hermitian"] == 1
    prog.run(dm)
    got = dm.to_numpy()
    want = ref.to_vectorised()
    assert max(np.abs(got.real - want.real).max(), np.abs(got.imag - want.imag).max()) <= TOL


@pytest.mark.parametrize("n", [2, 4, 7, 10])
def test_line_circuits(gpu_lib, n):
    check(gpu_lib, n, c1_line_circuit(n=n, n_gates=120), seed=n, tile_bits=12, min_contig_bits=2)


@pytest.mark.parametrize("contig", [1, 2])
def test_grid_circuit_eleven_qubits(gpu_lib, contig):
    ops = c2_grid_circuit(rows=1, cols=11, n_gates=300)
    check(gpu_lib, 11, ops, seed=11, tile_bits=12, min_contig_bits=contig)


@pytest.mark.parametrize("n,rows,tile_bits,contig", [(6, 2, 8, 1), (9, 1, 10, 1), (10, 2, 12, 1), (12, 2, 12, 1),
                                                     (12, 3, 12, 0)])
def test_relabelled_plans(gpu_lib, n, rows, tile_bits, contig):
    """relayout: between passes the state is stored under qubit relabellings,
    in two buffers; the result, in the caller's buffer under the original
    labelling, equals the oracle's.  Run twice on one handle (the second
    buffer is allocated once and reused)."""
    ops = c2_grid_circuit(rows=rows, cols=n // rows, n_gates=40 * n)
    R0 = hermitian_state(n, n + 100)
    ref = OracleDM(n)
    ref.set(R0)
    emulate(n, ops, ref)
    want = ref.to_vectorised()
    prog = gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(hermitian=True, relayout=True, tile_bits=tile_bits,
                                                             min_contig_bits=contig))
    say("relabelled n=%d ops=%d passes=%d" % (n, len(ops), prog.info()["n_passes"]))
    dm = gpu_lib.DensityMatrix(n)
    for rep in range(2):
        dm.from_numpy(np.ascontiguousarray(R0.T).reshape(-1))
        prog.run(dm)
        got = dm.to_numpy()
        assert max(np.abs(got.real - want.real).max(), np.abs(got.imag - want.imag).max()) <= TOL, rep


@pytest.mark.parametrize("tile_bits", [8, 10])
def test_all_to_all_small_tiles(gpu_lib, tile_bits):
    check(gpu_lib, 9, c3_all_to_all_circuit(n=9, n_gates=80), seed=3, tile_bits=tile_bits, min_contig_bits=2)


def test_named_channels_and_wide_gates(gpu_lib):
    from workloads import random_matrix_ops
    n = 8
    ops = random_matrix_ops(n, 8, seed=5, max_k=4, kraus=False)
    ops += [("depol1", (0,), (0.2,)), ("depol2", (1, 3), (0.3,)), ("amp", (2,), (0.4,)),
            ("gamp", (4,), (0.6, 0.3)), ("zz", (5, 0), (0.05,)), ("cz", (1, 7), ()), ("deph2", (2, 6), (0.1,))]
    ops += random_matrix_ops(n, 30, seed=6, max_k=2)
    check(gpu_lib, n, ops, seed=2, tile_bits=12, min_contig_bits=2)


def test_diagonal_tiles_of_passes_without_exchange(gpu_lib):
    """Regression: in a tile whose row and column group indices are equal
    the waves load each other's amplitudes through the transpose; in a pass
    without an LDS exchange only the kernel's barrier keeps a wave from
    storing the tile before the others have loaded it.  The 13-qubit grid
    circuit with three forced qubits has such passes; its result must equal
    the plan without Hermitian mode and be Hermitian to rounding (a stale
    load leaves errors of the size of one pass's change, about 1e-10)."""
    n = 13
    D = 1 << n
    ops = c2_grid_circuit(rows=1, cols=n, n_gates=2000)
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts()).run(dm)
    want = dm.to_numpy()
    prog = gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(hermitian=True, tile_bits=12, min_contig_bits=3))
    say("13q hermitian, %d passes" % prog.info()["n_passes"])
    dm.init_zero()
    prog.run(dm)
    got = dm.to_numpy()
    assert np.abs(got - want).max() <= 1e-12
    G = got.reshape(D, D)
    assert np.abs(G - G.conj().T).max() <= 1e-15
