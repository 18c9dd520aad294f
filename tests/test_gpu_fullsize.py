"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

14 qubits (4.3 GB): the oracle can follow a prefix of the grid circuit op by
op (about one second per op on the host), so the prefix is compared amplitude
by amplitude; the whole 9378-op circuit is checked through properties that
hold at any size and against the same circuit run one op per pass (no
fusion), on read-outs and on sampled amplitudes.

16 qubits (64 GiB, beyond the oracle's reach here): closed-form states (GHZ,
dephased |+>^16, diagonal-only circuits) and fused-versus-unfused agreement
on the all-to-all circuit.
"""
import math
import sys

import numpy as np
import pytest

import bench
from oracle.core import OracleDM
from oracle.emulator import emulate
from workloads import c2_grid_circuit, c3_all_to_all_circuit

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sample_amps(dm, idx):
    import torch
    b = dm.buffer.view(-1, 2)
    t = torch.as_tensor(idx, device=b.device)
    v = b[t].cpu().numpy()
    return v[:, 0] + 1j * v[:, 1]


@pytest.fixture(scope="module")
def grid14():
    return c2_grid_circuit(rows=2, cols=7, n_gates=2000)


def test_grid14_prefix_matches_oracle(gpu_lib, grid14):
    n = 14
    ops = grid14[:40]
    say("14q prefix of %d ops" % len(ops))
    prog = gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS))
    dm = gpu_lib.DensityMatrix(n)
    prog.run(dm)
    got = dm.to_numpy()
    ref = emulate(n, ops).to_vectorised()
    err = max(np.abs(got.real - ref.real).max(), np.abs(got.imag - ref.imag).max())
    say("max err", err)
    assert err <= TOL


def test_grid14_full_circuit_properties_and_unfused(gpu_lib, grid14):
    n = 14
    say("14q full circuit, fused (bench plan)")
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, grid14).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    tr = dm.trace()
    assert abs(tr - 1) <= TOL
    pur = dm.purity()
    assert 0 < pur <= 1
    z = dm.expec_z()
    assert np.all(np.abs(z) <= 1)
    probs = dm.probs()
    assert probs.min() >= -1e-12 and abs(probs.sum() - 1) <= TOL
    rng = np.random.default_rng(0)
    D = 1 << n
    r = rng.integers(0, D, 4000)
    c = rng.integers(0, D, 4000)
    a = sample_amps(dm, r + D * c)
    at = sample_amps(dm, c + D * r)
    assert np.abs(a - at.conj()).max() <= TOL            # Hermitian
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    zz = dm.expec_zz(pairs)
    say("14q unfused (one op per pass)")
    dm.init_zero()
    gpu_lib.Program(n, grid14).compile(gpu_lib.plan_opts(max_ops_per_pass=1)).run(dm)
    assert abs(dm.purity() - pur) <= TOL
    assert np.abs(dm.expec_z() - z).max() <= TOL
    assert np.abs(dm.expec_zz(pairs) - zz).max() <= TOL
    assert np.abs(sample_amps(dm, r + D * c) - a).max() <= TOL


def ghz_ops(n):
    ops = [("h", (0,), ())]
    for q in range(1, n):
        ops += [("h", (q,), ()), ("cz", (q - 1, q), ()), ("h", (q,), ())]
    return ops


def test_sixteen_qubit_closed_forms(gpu_lib):
    import torch
    n = 16
    if torch.cuda.get_device_properties(0).total_memory < 80 * 2 ** 30:
        pytest.skip("needs a GPU with more than 80 GiB")
    D = 1 << n
    say("16q GHZ")
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, ghz_ops(n)).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    corners = sample_amps(dm, [0, D - 1 + D * 0, 0 + D * (D - 1), (D - 1) * (D + 1)])
    assert np.abs(corners - 0.5).max() <= TOL
    rng = np.random.default_rng(1)
    idx = rng.integers(1, D * D - 1, 2000)
    idx = idx[(idx != D - 1) & (idx != D * (D - 1))]
    assert np.abs(sample_amps(dm, idx)).max() <= TOL
    assert abs(dm.purity() - 1) <= TOL
    assert np.abs(dm.expec_z()).max() <= TOL
    assert np.abs(dm.expec_zz([(0, 15), (3, 9), (7, 8)]) - 1).max() <= TOL

    say("16q |+>^16 dephased")
    p = 0.07
    ops = [("h", (q,), ()) for q in range(n)] + [("deph1", (q,), (p,)) for q in range(n)] * 2
    dm.init_zero()
    gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    for q in (0, 5, 15):
        codes = [0] * n
        codes[q] = 1
        assert abs(dm.expec_pauli(codes).real - (1 - 2 * p) ** 2) <= TOL
    assert abs(dm.purity() - ((1 + (1 - 2 * p) ** 4) / 2) ** n) <= TOL

    say("16q diagonal-only circuit keeps the diagonal")
    dm.init_product_diag(np.linspace(0.55, 0.95, n))
    before = dm.probs()
    ops = []
    for k in range(40):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        ops += [("rz", (a,), (float(rng.uniform(0, 6.3)),)), ("cz", (a, b), ()),
                ("zz", (b, a), (0.3,)), ("deph2", (a, b), (0.2,))]
    gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    assert np.abs(dm.probs() - before).max() <= TOL


def test_sixteen_qubit_all_to_all_fused_vs_unfused(gpu_lib):
    import torch
    n = 16
    if torch.cuda.get_device_properties(0).total_memory < 80 * 2 ** 30:
        pytest.skip("needs a GPU with more than 80 GiB")
    ops = c3_all_to_all_circuit(n=n, n_gates=500)
    D = 1 << n
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    rng = np.random.default_rng(2)
    idx = rng.integers(0, D * D, 3000)
    say("16q all-to-all, fused")
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    z, zz, pur, tr = dm.expec_z(), dm.expec_zz(pairs), dm.purity(), dm.trace()
    amp = sample_amps(dm, idx)
    assert abs(tr - 1) <= TOL and 0 < pur <= 1
    say("16q all-to-all, unfused")
    dm.init_zero()
    gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(max_ops_per_pass=1)).run(dm)
    assert np.abs(dm.expec_z() - z).max() <= TOL
    assert np.abs(dm.expec_zz(pairs) - zz).max() <= TOL
    assert abs(dm.purity() - pur) <= TOL
    assert np.abs(sample_amps(dm, idx) - amp).max() <= TOL
