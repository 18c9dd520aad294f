"""Trajectory kernel against the trajectory oracle (oracle/trajectories.py):
per trajectory, on the same uniforms, <Z_q>, squared norms and final states
agree to 1e-10 (the kernel and the oracle sum in different orders; a draw
could differ only if a uniform fell within rounding of an interval
boundary, which the seeded inputs do not).  Sizes span every thread layout
(1 to 13 qubits: several trajectories per wave, one per wave, several waves
per trajectory) and ragged trajectory counts."""
import sys

import numpy as np
import pytest

from oracle import trajectories as tj
from oracle.emulator import emulate
from workloads import c1_line_circuit, damped_layer_circuit, random_tp_ops, traj_grid_circuit, uniforms

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def mixed_ops(n, seed, count=30):
    """Random unitaries and Kraus maps plus named gates and channels."""
    ops = random_tp_ops(n, count, seed=seed, max_k=min(2, n))
    rng = np.random.default_rng(seed)
    for _ in range(count // 2):
        q = int(rng.integers(0, n))
        ops += [("su2", (q,), tuple(rng.standard_normal(4))), ("amp_t1", (q,), (0.5, 3.0)),
                ("depol1", (q,), (0.2,))]
        if n > 1:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            ops += [("cz", (a, b), ()), ("depol2", (a, b), (0.3,)), ("zz", (b, a), (0.2,))]
    return ops


@pytest.mark.parametrize("n,T", [(1, 5), (3, 37), (4, 300), (6, 70), (9, 11), (10, 9), (11, 5), (12, 3),
                                 (13, 3)])
def test_trajectories_match_oracle(gpu_lib, n, T):
    say("traj parity n=%d T=%d" % (n, T))
    ops = mixed_ops(n, seed=500 + n, count=24 if n < 12 else 10)
    prog = gpu_lib.Trajectories(n, ops).compile()
    U = uniforms(T, tj.n_channels(ops), seed=600 + n)
    out = prog.run(cuda(U), state=True)
    Z = out["z"].cpu().numpy()
    N = out["norm"].cpu().numpy()
    S = out["state"].cpu().numpy()
    for t in range(T):
        psi, _ = tj.run(n, ops, U[t])
        assert np.abs(Z[t] - tj.expec_z(psi)).max() <= TOL, (t, Z[t], tj.expec_z(psi))
        assert abs(N[t] - tj.norm2(psi)) <= TOL
        assert np.abs(S[t] - psi).max() <= TOL


@pytest.mark.parametrize("n,T", [(6, 40), (10, 24), (11, 12), (12, 8), (13, 4)])
def test_damping_runs_match_oracle(gpu_lib, n, T):
    """Runs of damping and dephasing draws taken with one reduction
    (trajectories of whole waves: 10 qubits and up, one to eight waves), with
    damping strong enough that many runs draw a jump and go member by member;
    below a wave (6 qubits) the runs are taken member by member.  Every
    trajectory against the oracle."""
    say("traj damping runs n=%d T=%d" % (n, T))
    ops = damped_layer_circuit(n, 3, seed=80 + n)
    prog = gpu_lib.Trajectories(n, ops).compile()
    U = uniforms(T, tj.n_channels(ops), seed=90 + n)
    out = prog.run(cuda(U), state=True)
    Z = out["z"].cpu().numpy()
    N = out["norm"].cpu().numpy()
    S = out["state"].cpu().numpy()
    for t in range(T):
        psi, _ = tj.run(n, ops, U[t])
        assert np.abs(Z[t] - tj.expec_z(psi)).max() <= TOL, (t, Z[t], tj.expec_z(psi))
        assert abs(N[t] - tj.norm2(psi)) <= TOL
        assert np.abs(S[t] - psi).max() <= TOL


def test_grid_circuit_sampled_trajectories(gpu_lib):
    """The 12-qubit grid circuit of the benchmark, 4096 trajectories in one
    launch; trajectories sampled across the batch against the oracle."""
    import torch
    n = 12
    ops = traj_grid_circuit()
    say("traj grid 12q: %d ops" % len(ops))
    prog = gpu_lib.Trajectories(n, ops).compile()
    T = 4096
    U = uniforms(T, tj.n_channels(ops))
    out = prog.run(cuda(U))
    torch.cuda.synchronize()
    Z = out["z"].cpu().numpy()
    N = out["norm"].cpu().numpy()
    assert np.abs(N - 1).max() <= 1e-10
    for t in (0, 1777, T - 1):
        psi, _ = tj.run(n, ops, U[t])
        assert np.abs(Z[t] - tj.expec_z(psi)).max() <= TOL, t


def test_mean_converges_to_density_matrix(gpu_lib):
    """The 6-qubit line circuit with stronger noise: the mean of 40000 GPU
    trajectories lies within 5 standard errors of the exact <Z_q> of the
    density-matrix oracle."""
    n = 6
    ops = [(k, q, (30 * p[0],) if k == "depol1" else p) for k, q, p in c1_line_circuit(n=n, n_gates=60)]
    prog = gpu_lib.Trajectories(n, ops).compile()
    U = cuda(uniforms(40000, tj.n_channels(ops), seed=77))
    say("traj convergence")
    Z = prog.run(U)["z"]
    mean, sem = gpu_lib.Trajectories.stats(Z)
    mean, sem = mean.cpu().numpy(), sem.cpu().numpy()
    exact = emulate(n, ops).expec_z()
    assert np.all(np.abs(mean - exact) <= 5 * sem), (mean, exact, sem)


def test_stats_kernel(gpu_lib):
    rng = np.random.default_rng(3)
    for T, m in ((1, 3), (2, 1), (1000, 7), (70001, 13)):
        x = rng.standard_normal((T, m)) * 3 + 1
        mean, sem = gpu_lib.Trajectories.stats(cuda(x))
        rm, rs = tj.estimate(x)
        assert np.abs(mean.cpu().numpy() - rm).max() <= 1e-12 * max(1, np.abs(rm).max())
        if T > 1:
            assert np.abs(sem.cpu().numpy() - rs).max() <= 1e-12 * rs.max()
        else:
            assert np.all(np.isinf(sem.cpu().numpy()))


def test_repeatable_and_edge_cases(gpu_lib):
    import torch
    n = 5
    ops = mixed_ops(n, seed=9)
    prog = gpu_lib.Trajectories(n, ops).compile()
    U = cuda(uniforms(513, tj.n_channels(ops), seed=10))
    a = prog.run(U)["z"].cpu().numpy()
    b = prog.run(U)["z"].cpu().numpy()
    assert np.array_equal(a, b)
    # count 0 does nothing; a prefix of the uniforms gives the same prefix of results
    prog.run(U[:0], count=0)
    c = prog.run(U[:100].contiguous())["z"].cpu().numpy()
    assert np.array_equal(c, a[:100])
    with pytest.raises(ValueError):
        prog.run(U.float())
    # a program without channels needs no uniforms
    gates = [op for op in ops if not tj.is_channel(op)]
    g = gpu_lib.Trajectories(n, gates).compile()
    z = g.run(None, count=3)["z"].cpu().numpy()
    psi, _ = tj.run(n, gates, [])
    assert np.abs(z - tj.expec_z(psi)).max() <= TOL
    torch.cuda.synchronize()


def test_silicon_device_stream_as_trajectories(gpu_lib):
    """The silicon preset's noisy stream (off-resonant drives, exchange
    crosstalk, dephasing, T1/T2 decay) as trajectories: sampled
    trajectories against the oracle, and the mean of 20000 within 5
    standard errors of the density-matrix oracle's <Z_q>."""
    from tests.test_presets import si_gates
    n = 6
    lib, _ = gpu_lib.Device.preset("silicon")
    ops = lib.insert_noise(si_gates(n, 40, 31))
    say("silicon trajectories: %d ops" % len(ops))
    prog = gpu_lib.Trajectories(n, ops).compile()
    T = 20000
    U = uniforms(T, tj.n_channels(ops), seed=91)
    out = prog.run(cuda(U))
    Z = out["z"]
    for t in (0, 4321, T - 1):
        psi, _ = tj.run(n, ops, U[t])
        assert np.abs(Z[t].cpu().numpy() - tj.expec_z(psi)).max() <= TOL, t
    mean, sem = gpu_lib.Trajectories.stats(Z)
    mean, sem = mean.cpu().numpy(), sem.cpu().numpy()
    exact = emulate(n, ops).expec_z()
    assert np.all(np.abs(mean - exact) <= 5 * sem + 1e-12), (mean, exact, sem)
