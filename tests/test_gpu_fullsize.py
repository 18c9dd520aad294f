"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

14 qubits (4.3 GB):
* the oracle follows the first 95 ops of the grid circuit live (the first
  SU(2) layer, its T1/T2 noise, the first CZ + depol2 layer and its ZZ
  crosstalk), compared amplitude by amplitude;
* the whole 9378-op circuit against the oracle's stored results
  (``tests/golden/grid14.json``, written by
  ``tests/golden/make_fullsize_goldens.py``): every <Z_i>, <Z_i Z_j>,
  probability, the purity and 8192 seeded amplitudes;
* the whole circuit in Hermitian mode against the same circuit planned
  without it, one op per pass (every tile computed, no fusion, no mirrored
  stores).

15 qubits (17.2 GB): the all-to-all circuit's generator against its stored
oracle results (``tests/golden/a2a15.json``).

16 qubits (64 GiB, beyond the oracle's reach here): closed-form states (GHZ,
dephased |+>^16, diagonal-only circuits) and fused-versus-unfused agreement
on the all-to-all circuit.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import bench
from oracle.core import OracleDM
from oracle.emulator import emulate
from workloads import c2_grid_circuit, c3_all_to_all_circuit

pytestmark = pytest.mark.gpu
TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
    ops = grid14[:95]
    kinds = {o[0] for o in ops}
    assert {"su2", "amp_t1", "deph_t2", "cz", "depol2", "zz"} <= kinds
    say("14q prefix of %d ops" % len(ops))
    prog = gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS))
    dm = gpu_lib.DensityMatrix(n)
    prog.run(dm)
    got = dm.to_numpy()
    del dm
    say("oracle on the host")
    ref = emulate(n, ops).to_vectorised()
    err = max(np.abs(got.real - ref.real).max(), np.abs(got.imag - ref.imag).max())
    say("max err", err)
    assert err <= TOL


def compare_with_golden(gpu_lib, dm, g):
    """Every stored read-out and sampled amplitude, element by element."""
    n = g["n"]
    D = 1 << n
    tr = dm.trace()
    assert abs(tr.real - g["trace"][0]) <= TOL and abs(tr.imag - g["trace"][1]) <= TOL
    assert abs(dm.purity() - g["purity"]) <= TOL
    assert np.abs(dm.expec_z() - np.asarray(g["expec_z"])).max() <= TOL
    pairs = [tuple(p) for p in g["pairs"]]
    assert len(pairs) == n * (n - 1) // 2
    assert np.abs(dm.expec_zz(pairs) - np.asarray(g["expec_zz"])).max() <= TOL
    probs = dm.probs()
    assert probs.shape == (D,)
    assert np.abs(probs - np.asarray(g["probs"])).max() <= TOL
    r = np.asarray(g["amp_rows"], dtype=np.int64)
    c = np.asarray(g["amp_cols"], dtype=np.int64)
    want = np.asarray(g["amp_re"]) + 1j * np.asarray(g["amp_im"])
    got = sample_amps(dm, r + D * c)      # rho_{rc} sits at r + 2^n c
    err = np.abs(got - want).max()
    say("max amplitude err", err)
    assert err <= TOL


def load_golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip("%s not written yet (tests/golden/make_fullsize_goldens.py %s)" % (path, name))
    with open(path) as f:
        return json.load(f)


def test_grid14_full_circuit_matches_oracle_golden(gpu_lib, grid14):
    g = load_golden("grid14")
    n = 14
    assert g["n"] == n and g["n_ops"] == len(grid14)
    say("14q full circuit (bench plan) vs stored oracle results")
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, grid14).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    compare_with_golden(gpu_lib, dm, g)


def test_all_to_all_15q_matches_oracle_golden(gpu_lib):
    g = load_golden("a2a15")
    n = 15
    ops = c3_all_to_all_circuit(n=n, n_gates=500)
    assert g["n"] == n and g["n_ops"] == len(ops)
    say("15q all-to-all (bench plan) vs stored oracle results")
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, ops).compile(gpu_lib.plan_opts(**bench.PLAN_OPTS)).run(dm)
    compare_with_golden(gpu_lib, dm, g)


def test_grid14_hermitian_mode_vs_full_unfused_plan(gpu_lib, grid14):
    n = 14
    assert bench.PLAN_OPTS["hermitian"]
    say("14q full circuit, fused (bench plan, Hermitian mode)")
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
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    zz = dm.expec_zz(pairs)
    say("14q one op per pass, every tile computed (no Hermitian mode)")
    dm.init_zero()
    gpu_lib.Program(n, grid14).compile(gpu_lib.plan_opts(max_ops_per_pass=1, hermitian=False)).run(dm)
    # both triangles were computed independently here, so Hermiticity is a check
    b = sample_amps(dm, r + D * c)
    bt = sample_amps(dm, c + D * r)
    assert np.abs(b - bt.conj()).max() <= TOL
    assert abs(dm.purity() - pur) <= TOL
    assert np.abs(dm.expec_z() - z).max() <= TOL
    assert np.abs(dm.expec_zz(pairs) - zz).max() <= TOL
    assert np.abs(b - a).max() <= TOL


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
