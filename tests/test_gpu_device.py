"""Noise inserted by the device layer, run on the GPU density-matrix path,
against the oracle's noise insertion run on the density-matrix oracle."""
import sys

import numpy as np
import pytest

from oracle import device as dv
from oracle.emulator import emulate
from tests.test_device_cpu import lib_device
from workloads import c2_grid_circuit

pytestmark = pytest.mark.gpu


def test_device_stream_on_the_density_matrix(gpu_lib):
    n = 8
    ideal = [op for op in c2_grid_circuit(rows=2, cols=4, n_gates=160) if op[0] in ("su2", "cz")]
    ref = dv.Device(n)
    ref.set_gate("su2", 0.05, 1e-3, 5e-4)
    ref.set_gate("cz", 0.5, 5e-3, 1e-3)
    ref.set_passive([100.0] * n, [50.0] * n)
    ref.set_crosstalk([(a, a + 1) for a in range(7) if a != 3] + [(a, a + 4) for a in range(4)], 0.01)
    noisy = lib_device(gpu_lib, ref).insert_noise(ideal)
    print("device stream: %d ops" % len(noisy), flush=True)
    sys.stdout.flush()
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, noisy).compile().run(dm)
    want = emulate(n, dv.insert_noise(ref, ideal))
    assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10
    assert abs(dm.purity() - want.purity()) <= 1e-10
