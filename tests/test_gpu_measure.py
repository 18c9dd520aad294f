"""Measurement kernels against the measurement oracle (oracle/measure.py):
outcomes, weights and collapsed states of projective Z and parity
measurements, and sampled shots, on the same states and uniforms."""
import sys

import numpy as np
import pytest

from oracle import measure as ms
from oracle.emulator import emulate
from workloads import c2_grid_circuit, random_tp_ops

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state_pair(gpu_lib, n, seed):
    ops = random_tp_ops(n, 3 * n, seed=seed, max_k=min(2, n))
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, ops).compile().run(dm)
    return dm, emulate(n, ops)


def check_shots(got, probs, U, n):
    """Shots of the library against the oracle's draw on the same
    probabilities: the running sums are rounded in different orders (the
    oracle left to right, the kernel per thread run and then chained), so a
    shot may differ only where u W lies within rounding of a boundary of the
    oracle's running sums, and never lands on a zero-probability state."""
    ref = ms.sample(probs, U)
    p = np.maximum(np.asarray(probs, dtype=np.float64), 0)
    cum = np.cumsum(p)
    for s in np.nonzero(got != ref)[0]:
        thr = U[s] * cum[-1]
        assert np.min(np.abs(cum - thr)) <= 1e-12 * cum[-1], (s, got[s], ref[s])
    assert got.min() >= 0 and got.max() < (1 << n)
    assert np.all(p[got] > 0)
    return int(np.count_nonzero(got != ref))


def safe_u(w, m):
    """A uniform well inside outcome m's interval."""
    W = w[0] + w[1]
    return 0.5 * w[0] / W if m == 0 else (w[0] + 0.5 * w[1]) / W


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_measure_z_matches_oracle(gpu_lib, n):
    for q in range(n):
        for m in (0, 1):
            say("measure_z n=%d q=%d m=%d" % (n, q, m))
            dm, ref = state_pair(gpu_lib, n, 40 + n)
            w_ref = [float(np.real(np.diag(ref.R))[((np.arange(1 << n) >> q) & 1) == k].sum()) for k in (0, 1)]
            if w_ref[m] < 1e-9:
                continue
            u = safe_u(w_ref, m)
            out, w = dm.measure_z(q, u)
            out_r, wr = ms.measure_z(ref, q, u)
            assert out == out_r == m
            assert abs(w - wr[m]) <= TOL
            assert np.abs(dm.to_numpy() - ref.to_vectorised()).max() <= TOL
            assert abs(dm.trace() - 1) <= TOL


@pytest.mark.parametrize("n,q0,q1", [(2, 0, 1), (3, 2, 0), (5, 1, 4), (6, 5, 3)])
def test_measure_parity_matches_oracle(gpu_lib, n, q0, q1):
    for m in (0, 1):
        say("measure_parity n=%d (%d,%d) m=%d" % (n, q0, q1, m))
        dm, ref = state_pair(gpu_lib, n, 70 + n)
        x = np.arange(1 << n)
        par = ((x >> q0) ^ (x >> q1)) & 1
        d = np.real(np.diag(ref.R))
        w_ref = [float(d[par == 1].sum()), float(d[par == 0].sum())]
        u = safe_u(w_ref, m)
        out, w = dm.measure_parity(q0, q1, u)
        out_r, wr = ms.measure_parity(ref, q0, q1, u)
        assert out == out_r == m
        assert abs(w - wr[m]) <= TOL
        assert np.abs(dm.to_numpy() - ref.to_vectorised()).max() <= TOL


def test_certain_outcomes_and_errors(gpu_lib):
    dm = gpu_lib.DensityMatrix(3)
    for u in (0.0, 0.5, 0.999999):
        assert dm.measure_z(1, u) == (0, 1.0)
        assert dm.measure_parity(0, 2, u)[0] == 1          # |000> has even parity
    assert np.abs(dm.to_numpy()[0] - 1) <= TOL
    with pytest.raises(gpu_lib.VQDError):
        dm.measure_z(3, 0.5)
    with pytest.raises(gpu_lib.VQDError):
        dm.measure_z(0, 1.0)
    with pytest.raises(gpu_lib.VQDError):
        dm.measure_parity(1, 1, 0.5)


@pytest.mark.parametrize("n,shots", [(1, 100), (4, 3000), (8, 20000), (10, 4097)])
def test_sampling_matches_oracle(gpu_lib, n, shots):
    import torch
    say("sample n=%d shots=%d" % (n, shots))
    dm, ref = state_pair(gpu_lib, n, 90 + n)
    U = np.random.default_rng(n).random(shots)
    got = dm.sample(torch.as_tensor(U, device="cuda")).cpu().numpy().astype(np.int64)
    # on the library's own probabilities and on the oracle's
    check_shots(got, dm.probs(), U, n)
    check_shots(got, ref.probs(), U, n)


@pytest.mark.parametrize("n", [1, 3, 8, 9, 12, 14])
def test_sampling_exact_sums(gpu_lib, n):
    """Diagonals of dyadic probabilities (multiples of 2^-24, about a third of
    them zero): every running sum is exact in any order, so the shots equal
    the oracle's one for one, including uniforms that hit a boundary exactly
    and the top end (the last state with nonzero probability).  Sizes span
    one thread's run (below 256 states) to 64 states per thread."""
    import torch
    say("sample exact n=%d" % n)
    D = 1 << n
    rng = np.random.default_rng(300 + n)
    k = rng.integers(0, 64, size=D).astype(np.float64)
    k[rng.random(D) < 0.35] = 0.0
    k[-1] = 0.0
    k[0] = max(k[0], 1.0)
    probs = k / 2.0 ** 24
    dm = gpu_lib.DensityMatrix(n)
    dm.buffer.zero_()
    # amp[r + 2^n c] = rho[r][c]: the diagonal's real parts at 2 x (D + 1)
    idx = torch.arange(D, device="cuda") * (2 * (D + 1))
    dm.buffer[idx] = torch.as_tensor(probs, device="cuda")
    torch.cuda.synchronize()
    cum = np.cumsum(probs)
    W = cum[-1]
    edges = cum[:-1][probs[1:] > 0] / W          # exact boundaries
    U = np.concatenate([rng.random(20000), edges[:500], [0.0, np.nextafter(1.0, 0.0)]])
    got = dm.sample(torch.as_tensor(U, device="cuda")).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, ms.sample(probs, U))
    assert np.all(probs[got] > 0)


def test_fourteen_qubit_collapse_and_shots(gpu_lib):
    """The 14-qubit grid-circuit state: collapse keeps exactly the support
    (sampled elements against a copy taken before), <Z_q> becomes +-1, the
    trace 1; a million shots equal the oracle's draw on the same
    probabilities (up to rounding at interval boundaries)."""
    import torch
    n = 14
    say("14q collapse")
    dm = gpu_lib.DensityMatrix(n)
    gpu_lib.Program(n, c2_grid_circuit(rows=2, cols=7, n_gates=200)).compile().run(dm)
    probs = dm.probs()
    U = np.random.default_rng(5).random(1 << 20)
    got = dm.sample(torch.as_tensor(U, device="cuda")).cpu().numpy().astype(np.int64)
    assert check_shots(got, probs, U, n) <= 4
    before = dm.buffer.clone()
    q = 9
    z = dm.expec_z()[q]
    w0 = 0.5 * (1 + z)
    out, w = dm.measure_z(q, 0.5 * w0)
    assert out == 0 and abs(w - w0) <= 1e-12
    assert abs(dm.expec_z()[q] - 1) <= TOL and abs(dm.trace() - 1) <= TOL
    idx = torch.as_tensor(np.random.default_rng(6).integers(0, 4 ** n, 200000), device="cuda")
    r, c = idx & ((1 << n) - 1), idx >> n
    keep = (((r >> q) & 1) == 0) & (((c >> q) & 1) == 0)
    b = before.view(torch.complex128)[idx] if before.dtype != torch.complex128 else before[idx]
    a = dm.buffer.view(torch.complex128)[idx] if dm.buffer.dtype != torch.complex128 else dm.buffer[idx]
    expect = torch.where(keep, b / w, torch.zeros_like(b))
    assert torch.max(torch.abs(a - expect)).item() <= 1e-12
