"""Trajectory planner on the CPU: plans exported by the library
(vqd_traj_export) are executed by tests/_traj_emu.py and compared, trajectory
by trajectory, with the trajectory oracle on the same uniforms."""
import numpy as np
import pytest

from oracle import trajectories as tj
from tests import _traj_emu as emu
from workloads import (c1_line_circuit, c2_grid_circuit, c3_all_to_all_circuit, damped_layer_circuit,
                       random_tp_ops, uniforms)


def check_plan(vqd, n, ops, T=8, seed=0, tol=1e-12):
    t = vqd.Trajectories(n, ops).plan()
    plan = emu.parse(t.export())
    nch = tj.n_channels(ops)
    info = t.info()
    assert info["n_channels"] == nch == plan["n_channels"]
    assert info["n_mixed"] + info["n_general"] == nch
    U = uniforms(T, nch, seed=seed)
    Z, N, order = emu.run(plan, U)
    assert order == list(range(nch))          # channels met in channel order
    Zr, Nr = tj.run_many(n, ops, U)
    assert np.abs(Z - Zr).max() <= tol, np.abs(Z - Zr).max()
    assert np.abs(N - Nr).max() <= tol
    return t, plan


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_random_unitaries_and_kraus_maps(vqd_host, n):
    ops = random_tp_ops(n, 40, seed=200 + n, max_k=min(2, n))
    check_plan(vqd_host, n, ops)


@pytest.mark.parametrize("n", [2, 5])
def test_three_and_four_qubit_gates(vqd_host, n):
    """Gates on up to four qubits (k <= n) among channels."""
    rng = np.random.default_rng(n)
    ops = []
    for i in range(12):
        k = int(rng.integers(1, min(4, n) + 1))
        ops += random_tp_ops(n, 1, seed=300 + i, max_k=min(2, n), p_channel=1.0)
        tg = tuple(int(x) for x in rng.choice(n, size=k, replace=False))
        Q, _ = np.linalg.qr(rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k)))
        ops.append(("matrix", tg, (Q,)))
    check_plan(vqd_host, n, ops)


def test_named_gates_and_channels(vqd_host):
    n = 5
    ops = [("h", (0,), ()), ("x", (1,), ()), ("y", (2,), ()), ("z", (3,), ()), ("rx", (4,), (0.3,)),
           ("ry", (0,), (1.1,)), ("rz", (1,), (2.2,)), ("su2", (2,), (0.1, -0.7, 0.4, 0.2)),
           ("cz", (0, 3), ()), ("cphase", (4, 1), (0.6,)), ("xx", (2, 0), (0.9,)), ("zz", (3, 4), (0.05,)),
           ("depol1", (0,), (0.2,)), ("depol2", (1, 3), (0.3,)), ("deph1", (2,), (0.25,)),
           ("deph2", (4, 0), (0.1,)), ("amp", (1,), (0.4,)), ("gamp", (3,), (0.6, 0.3)),
           ("bitflip1", (4,), (0.2,)), ("bitflip2", (2, 1), (0.3,)), ("amp_t1", (0,), (0.5, 2.0)),
           ("deph_t2", (3,), (0.5, 1.0)), ("gamp_t1", (2,), (0.9, 0.5, 2.0)), ("depol_t1", (4,), (0.3, 2.0)),
           ("deph_t2s", (1,), (0.4, 1.5)), ("rabi", (3,), (1.7, 0.9, -0.6, 1.3)),
           ("offres", (0,), (1.0, 2.0, 0.7)), ("crz", (1, 4), (0.8,)), ("parity_decay", (2, 0), ())]
    _, plan = check_plan(vqd_host, n, ops * 3, T=24)
    kinds = set(int(k) for k in plan["ops"]["kind"])
    assert kinds >= {emu.TOP_MAT, emu.TOP_DTHR, emu.TOP_DREG, emu.TOP_DMIX, emu.TOP_DRM, emu.TOP_MIX, emu.TOP_KRAUS}


def test_workload_circuits(vqd_host):
    check_plan(vqd_host, 6, c1_line_circuit(), T=3)
    check_plan(vqd_host, 6, c2_grid_circuit(rows=2, cols=3, n_gates=60), T=3)
    check_plan(vqd_host, 7, c3_all_to_all_circuit(n=7, n_gates=40), T=3)


def test_gate_only_and_empty_programs(vqd_host):
    ops = [op for op in c1_line_circuit(n=4, n_gates=20) if not tj.is_channel(op)]
    check_plan(vqd_host, 4, ops, T=1)
    t = vqd_host.Trajectories(3).plan()
    plan = emu.parse(t.export())
    Z, N, _ = emu.run(plan, np.zeros((2, 0)))
    assert np.array_equal(Z, np.ones((2, 3))) and np.array_equal(N, np.ones(2))


def test_phase_layouts_are_permutations(vqd_host):
    n = 9
    t = vqd_host.Trajectories(n, c2_grid_circuit(rows=3, cols=3, n_gates=200)).plan()
    plan = emu.parse(t.export())
    for ph in plan["phases"]:
        qs = list(ph["reg"]) + list(ph["thr"][:n - 4])
        assert sorted(int(q) for q in qs) == list(range(n))
    # fusion and reordering keep the plan well below one phase per op
    assert len(plan["phases"]) < len(plan["ops"])


def test_errors(vqd_host):
    v = vqd_host
    with pytest.raises(v.VQDError):
        v.Trajectories(0)
    with pytest.raises(v.VQDError):
        v.Trajectories(14)
    t = v.Trajectories(3)
    with pytest.raises(v.VQDError):                # not unitary
        t.add(("matrix", (0,), (np.array([[1, 0], [0, 2]]),)))
    with pytest.raises(v.VQDError):                # too many Kraus operators
        t.add(("kraus", (0,), tuple(np.eye(2) / np.sqrt(17) for _ in range(17))))
    with pytest.raises(v.VQDError):                # Kraus maps on at most two qubits
        t.add(("kraus", (0, 1, 2), (np.eye(8),)))
    with pytest.raises(v.VQDError):                # duplicate target
        t.add(("cz", (1, 1), ()))
    with pytest.raises(v.VQDError):                # bad probability
        t.add(("depol1", (0,), (1.5,)))
    with pytest.raises(v.VQDError):                # bad op inside a batch of named ops: all or nothing
        t.extend([("h", (0,), ()), ("depol1", (5,), (0.1,))])
    assert t.info()["n_ops"] == 0
    with pytest.raises(v.VQDError):                # not planned yet
        t.export()


def test_inline_channel_coefficients_match_the_pool(vqd_host):
    """One-qubit two-operator channels carry the numbers of their draw in the
    descriptor (the kernel's inline path); they must equal the pool's full
    form: a mixed-unitary channel's running sums and its operators'
    diagonals, a damping channel's Gram diagonals and K_0's diagonal.  Other
    mixed-unitary channels whose operator 0 is the identity carry their
    first running sum and total."""
    from workloads import traj_grid_circuit
    t = vqd_host.Trajectories(12, traj_grid_circuit())
    t.plan()
    plan = emu.parse(t.export())
    pool = plan["pool"]
    seen = {emu.TOP_MIX: 0, emu.TOP_KRAUS: 0, "identity_first": 0}
    for op in plan["ops"]:
        if not int(op["inl"]):
            continue
        kind, m, cf = int(op["kind"]), int(op["mat"]), op["cf"]
        if int(op["inl"]) == 2:
            # a mixed-unitary channel whose operator 0 is the identity: the
            # first running sum and the total
            nk = int(op["nk"])
            d = 1 << bin(int(op["mask"])).count("1")
            assert kind == emu.TOP_MIX and cf[0] == pool[m].real and cf[1] == pool[m + nk - 1].real
            assert np.array_equal(pool[m + nk:m + nk + d * d], np.eye(d).reshape(-1))
            seen["identity_first"] += 1
            continue
        assert bin(int(op["mask"])).count("1") == 1 and int(op["nk"]) == 2
        seen[kind] += 1
        if kind == emu.TOP_MIX:
            assert cf[0] == pool[m].real and cf[1] == pool[m + 1].real
            for j in range(2):
                U = pool[m + 2 + 4 * j:m + 6 + 4 * j]
                assert U[1] == 0 and U[2] == 0 and U[0].imag == 0 and U[3].imag == 0
                assert (cf[2 + 2 * j], cf[3 + 2 * j]) == (U[0].real, U[3].real)
        else:
            assert kind == emu.TOP_KRAUS and int(op["gdiag"])
            for i in range(2):
                G = pool[m + 4 * i:m + 4 * i + 4]
                assert (cf[2 * i], cf[2 * i + 1]) == (G[0].real, G[3].real)
            K0 = pool[m + 8:m + 12]
            assert K0[1] == 0 and K0[2] == 0 and (cf[4], cf[5]) == (K0[0].real, K0[3].real)
    # the grid circuit's dephasing and damping channels all take the inline
    # path, its two-qubit depolarising channels the identity-first one
    assert seen[emu.TOP_MIX] >= 2000 and seen[emu.TOP_KRAUS] >= 2000 and seen["identity_first"] >= 500


def test_inline_runs_are_marked(vqd_host):
    """Runs of one-qubit channels with inline coefficients carry their length
    on their first op: members inline, in one phase, at most 8 ops and 4
    damping channels, at least 2 of them, and mixed-unitary members with
    diagonal entries of magnitude 1 up to rounding (they must not move
    populations).  In
    the 12-qubit grid circuit every damping channel is in such a run."""
    from workloads import traj_grid_circuit
    for n, ops in ((12, traj_grid_circuit()), (11, damped_layer_circuit(11, 3, seed=5)), (6, damped_layer_circuit(6, 2, seed=6))):
        t = vqd_host.Trajectories(n, ops)
        t.plan()
        plan = emu.parse(t.export())
        O = plan["ops"]
        covered = np.zeros(len(O), dtype=bool)
        for ph in plan["phases"]:
            ob, oe = int(ph["ob"]), int(ph["oe"])
            for i in range(ob, oe):
                k = int(O[i]["grp"])
                if not k:
                    continue
                assert 2 <= k <= 8 and i + k <= oe and not covered[i]
                kinds = [int(m["kind"]) for m in O[i:i + k]]
                assert all(int(m["inl"]) == 1 for m in O[i:i + k])
                assert 2 <= kinds.count(emu.TOP_KRAUS) <= 4
                for m in O[i:i + k]:
                    if int(m["kind"]) == emu.TOP_MIX:
                        assert np.all(np.abs(np.abs(m["cf"][2:6]) - 1.0) <= 1e-15)
                assert all(int(m["grp"]) == 0 for m in O[i + 1:i + k])
                covered[i:i + k] = True
        damp = np.array([int(o["kind"]) == emu.TOP_KRAUS and int(o["inl"]) == 1 for o in O])
        assert damp.any()
        if n == 12:
            assert covered[damp].all()


@pytest.mark.parametrize("n,T", [(10, 6), (12, 4)])
def test_grouped_draws_match_oracle(vqd_host, n, T):
    """The grouped draw rule (every damping weight of a run from the run's
    input populations, one normalisation at the end) gives the oracle's
    trajectories on the same uniforms, through both of its paths: runs with
    no jump, and runs where a jump sends the members one by one."""
    ops = damped_layer_circuit(n, 3, seed=40 + n)
    t = vqd_host.Trajectories(n, ops)
    t.plan()
    plan = emu.parse(t.export())
    U = uniforms(T, tj.n_channels(ops), seed=70 + n)
    st = {}
    Z, N, order = emu.run(plan, U, groups=True, stats=st)
    assert order == list(range(tj.n_channels(ops)))
    Zr, Nr = tj.run_many(n, ops, U)
    assert np.abs(Z - Zr).max() <= 1e-12
    assert np.abs(N - Nr).max() <= 1e-12
    assert st["grouped"] > 0 and st["fallback"] > 0, st
