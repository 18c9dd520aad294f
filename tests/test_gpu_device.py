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


def test_superconducting_preset_with_readout(gpu_lib):
    """The superconducting preset end to end on the GPU: thermal initial
    state, the noisy circuit, read-out noise, a projective measurement of
    every qubit and the noise after it, against the oracle."""
    from oracle import measure as om
    from tests.test_presets import oracle_superconducting, sc_gates
    n = 6
    dev, p0 = gpu_lib.Device.preset("superconducting")
    ref, rp0 = oracle_superconducting()
    gates = sc_gates(n, 150, 21)
    noisy = dev.insert_noise(gates) + dev.readout_noise(list(range(n)), 0)
    want_ops = dv.insert_noise(ref, gates) + dv.readout_noise(ref, list(range(n)), 0)
    print("superconducting preset: %d ops" % len(noisy), flush=True)
    dm = gpu_lib.DensityMatrix(n)
    dm.init_product_diag(p0)
    gpu_lib.Program(n, noisy).compile().run(dm)
    from oracle.core import OracleDM
    want = OracleDM(n)
    want.init_product_diag(rp0)
    emulate(n, want_ops, want)
    assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10
    U = np.random.default_rng(5).random(n)
    for q in range(n):
        m, w = dm.measure_z(q, float(U[q]))
        mr, wr = om.measure_z(want, q, float(U[q]))
        assert m == mr and abs(w - wr[mr]) <= 1e-10
    post = dev.readout_noise(list(range(n)), 1)
    gpu_lib.Program(n, post).compile().run(dm)
    emulate(n, dv.readout_noise(ref, list(range(n)), 1), want)
    assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10


def test_off_resonant_driving_on_the_density_matrix(gpu_lib):
    """Off-resonant driving (Sec. 3.3) with silicon-like qubit and Rabi
    frequencies (Sec. 7 table; angular, per microsecond): x and y rotations
    of angle-scaled duration drive the passive qubits, on the GPU against the
    oracle, in the default and the Hermitian plan."""
    n = 6
    two_pi = 2 * np.pi
    freq = [two_pi * f for f in (15.62e3, 15.88e3, 16.3e3, 16.1e3, 15.9e3, 15.69e3)]
    ref = dv.Device(n)
    for k in ("rx", "ry"):
        ref.set_gate(k, 0.1, 0.0, 1e-4)
        ref.set_angle_scaling(k, True, True)
    ref.set_gate("cz", 0.2, 0.0, 2e-3)
    ref.set_passive([1e4] * n, [14.0, 21.1, 40.1, 37.2, 44.7, 26.7])
    # frequency differences divided by 100 (Omega / Delta of order 1 instead
    # of ~0.02), so that the detuned drives move the bystanders visibly
    ref.set_off_resonant([two_pi * 5.0] * n, [f / 100.0 for f in freq])
    rng = np.random.default_rng(11)
    ideal = []
    for _ in range(60):
        if rng.random() < 0.25:
            a = int(rng.integers(n - 1))
            ideal.append(("cz", (a, a + 1), ()))
        else:
            ideal.append((str(rng.choice(["rx", "ry"])), (int(rng.integers(n)),), (float(rng.uniform(-np.pi, np.pi)),)))
    noisy = lib_device(gpu_lib, ref).insert_noise(ideal)
    assert sum(1 for k, _, _ in noisy if k == "offres") > 50
    print("off-resonant stream: %d ops" % len(noisy), flush=True)
    want = emulate(n, dv.insert_noise(ref, ideal))
    for opts in (None, gpu_lib.plan_opts(hermitian=True, tile_bits=8, min_contig_bits=1)):
        dm = gpu_lib.DensityMatrix(n)
        gpu_lib.Program(n, noisy).compile(opts).run(dm)
        assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10


def test_silicon_preset_on_the_density_matrix(gpu_lib):
    """The silicon preset (serial gates, off-resonant driving, exchange
    crosstalk, per-qubit and per-pair dephasing) on the GPU against the
    oracle's device built from the printed table."""
    from tests.test_presets import oracle_silicon, si_gates
    n = 6
    lib, _ = gpu_lib.Device.preset("silicon")
    ref, _ = oracle_silicon()
    ideal = si_gates(n, 80, 21)
    noisy = lib.insert_noise(ideal)
    print("silicon stream: %d ops" % len(noisy), flush=True)
    want = emulate(n, dv.insert_noise(ref, ideal))
    # the Hermitian plan first (every op here preserves Hermiticity)
    herm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, noisy).compile(gpu_lib.plan_opts(hermitian=True, tile_bits=8, min_contig_bits=1)).run(herm)
    assert np.abs(herm.to_numpy() - want.to_vectorised()).max() <= 1e-10
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, noisy).compile().run(dm)
    assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10
    # parity read-out of the two edge pairs (eq. projmeas, eq. m)
    from oracle import measure as om
    for (q0, q1), u in (((0, 1), 0.3), ((4, 5), 0.8)):
        gpu_lib.Program(n, lib.parity_readout_noise(q0, q1, 0)).compile().run(dm)
        emulate(n, dv.parity_readout_noise(ref, q0, q1, 0), want)
        m, w = dm.measure_parity(q0, q1, u)
        mr, wr = om.measure_parity(want, q0, q1, u)
        assert m == mr and abs(w - wr[mr]) <= 1e-10
        gpu_lib.Program(n, lib.parity_readout_noise(q0, q1, 1)).compile().run(dm)
        emulate(n, dv.parity_readout_noise(ref, q0, q1, 1), want)
        assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10


def test_trapped_ion_preset_with_readout(gpu_lib):
    """The trapped-ion preset end to end on the GPU: initialisation errors,
    the noisy circuit, the bit-flip read-out of two ions and their
    projective measurements, against the oracle."""
    from oracle import measure as om
    from oracle.core import OracleDM
    from tests.test_device_oracle import random_gates
    from tests.test_presets import oracle_trapped_ion
    n = 8
    dev, p0 = gpu_lib.Device.preset("trapped_ion")
    ref, rp0 = oracle_trapped_ion()
    gates = random_gates(n, 60, 23)
    noisy = dev.insert_noise(gates) + dev.readout_noise([2, 6], 0)
    print("trapped-ion preset: %d ops" % len(noisy), flush=True)
    dm = gpu_lib.DensityMatrix(n)
    dm.init_product_diag(p0)
    gpu_lib.Program(n, noisy).compile().run(dm)
    want = OracleDM(n)
    want.init_product_diag(rp0)
    emulate(n, dv.insert_noise(ref, gates) + dv.readout_noise(ref, [2, 6], 0), want)
    assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10
    for q, u in ((2, 0.4), (6, 0.9)):
        m, w = dm.measure_z(q, u)
        mr, wr = om.measure_z(want, q, u)
        assert m == mr and abs(w - wr[mr]) <= 1e-10
    assert np.abs(dm.to_numpy() - want.to_vectorised()).max() <= 1e-10
