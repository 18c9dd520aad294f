"""The read-out entry point for callers that cannot allocate:
vqd_calc_expec_z_noalloc (no handle, static device scratch) against the
handle-based vqd_calc_expec_z_dev on the same states, two calls in a row,
the second on a smaller state (the scratch keeps the first call's partials,
which the second must not see).  Values must be bit-identical (same kernels,
same summation order) and within 1e-10 of the CPU oracle."""
import sys

import numpy as np
import pytest

from oracle.emulator import emulate
from workloads import c1_line_circuit, c2_grid_circuit

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_expec_z_matches_handle_readout_twice(gpu_lib):
    import torch
    cases = [(12, c2_grid_circuit(rows=2, cols=6, n_gates=60)), (5, c1_line_circuit(n=5, n_gates=60))]
    for n, ops in cases:
        say("no-alloc <Z> on %d qubits" % n)
        dm = gpu_lib.DensityMatrix(n)
        gpu_lib.Program(n, ops).compile().run(dm)
        ref_dev = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        dm.expec_z_dev(ref_dev)
        got = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        gpu_lib.calc_expec_z_noalloc(dm.buffer, n, got)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref_dev.cpu().numpy()
        assert np.array_equal(g, r), (n, g, r)
        want = emulate(n, ops).expec_z()
        assert np.abs(g - want).max() <= TOL
        dm.close()


def test_noalloc_rejects_bad_arguments(gpu_lib):
    import torch
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    amps = torch.zeros(2 * 4 ** 2, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        gpu_lib.calc_expec_z_noalloc(amps, 3, out)          # buffer too small for n = 3
    L = gpu_lib.lib()
    import ctypes
    assert L.vqd_calc_expec_z_noalloc(ctypes.c_void_p(amps.data_ptr()), 17, None,
                                      ctypes.c_void_p(out.data_ptr())) == -2
    assert L.vqd_calc_expec_z_noalloc(None, 2, None, ctypes.c_void_p(out.data_ptr())) == -1
