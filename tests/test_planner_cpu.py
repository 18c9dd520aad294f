"""Planner checks on the CPU: plans exported by the library are executed by a
numpy emulation of the pass kernel (tests/_plan_emu.py) and compared with the
oracle.  Covers fusion on/off, one op per pass, tile sizes from the 4-bit
minimum to 12 bits, tiles without contiguous low bits, phantom bits (n = 1),
wide (3- and 4-qubit) unitary blocks, diagonal ops inside and outside the
tile, and non-Hermitian starting states (a missing conjugate shows)."""
import numpy as np
import pytest

from oracle.core import OracleDM
from oracle.emulator import emulate
from tests import _plan_emu as emu
from workloads import (c1_line_circuit, c2_grid_circuit, c3_all_to_all_circuit,
                       random_matrix_ops)


def start_state(n, seed):
    rng = np.random.default_rng(seed)
    D = 1 << n
    R = (rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))) / D
    return R


def run_both(vqd, n, ops, seed=0, **opts):
    R0 = start_state(n, seed)
    dm = OracleDM(n)
    dm.set(R0)
    emulate(n, ops, dm)
    ref = dm.to_vectorised()
    prog = vqd.Program(n, ops)
    prog.plan(vqd.plan_opts(**opts))
    plan = emu.parse(prog.export())
    got = emu.run(plan, np.ascontiguousarray(R0.T).reshape(-1))
    info = prog.info()
    return got, ref, info


def assert_close(got, ref, tol=1e-12):
    err = np.abs(got - ref).max()
    assert err <= tol * max(1.0, np.abs(ref).max()), err


@pytest.mark.parametrize("n", [4, 6])
def test_c1_circuit_default_plan(vqd_host, n):
    ops = c1_line_circuit(n=n, n_gates=80)
    got, ref, info = run_both(vqd_host, n, ops)
    assert_close(got, ref)
    assert info["n_passes"] >= 1


@pytest.mark.parametrize("tile_bits,contig,max_ops,fuse", [
    (13, 3, 0, True), (12, 3, 0, False), (8, 3, 0, True), (6, 0, 0, True),
    (4, 0, 0, True), (12, 3, 1, True), (10, 2, 3, True), (7, 7, 0, True)])
@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_random_matrices_all_plans(vqd_host, n, tile_bits, contig, max_ops, fuse):
    ops = random_matrix_ops(n, 30, seed=7 * n + tile_bits, max_k=2)
    if n >= 2 and tile_bits >= 8:
        ops += random_matrix_ops(n, 6, seed=3, max_k=min(4, n), kraus=False)
    got, ref, info = run_both(vqd_host, n, ops, seed=n, tile_bits=tile_bits,
                              min_contig_bits=contig, max_ops_per_pass=max_ops,
                              fuse_blocks=fuse)
    assert_close(got, ref)
    if max_ops == 1:
        assert info["n_passes"] == len(ops)


@pytest.mark.parametrize("tile_bits", [6, 8, 12])
def test_diagonal_ops_inside_and_outside_tile(vqd_host, tile_bits):
    n = 6
    rng = np.random.default_rng(tile_bits)
    ops = []
    for _ in range(60):
        r = rng.integers(0, 7)
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        if r == 0:
            ops.append(("rz", (a,), (float(rng.uniform(0, 6.3)),)))
        elif r == 1:
            ops.append(("cz", (a, b), ()))
        elif r == 2:
            ops.append(("zz", (a, b), (float(rng.uniform(0, 1)),)))
        elif r == 3:
            ops.append(("deph1", (a,), (float(rng.uniform(0, 0.5)),)))
        elif r == 4:
            ops.append(("deph2", (a, b), (float(rng.uniform(0, 0.7)),)))
        elif r == 5:
            ops.append(("ry", (a,), (float(rng.uniform(0, 6.3)),)))
        else:
            ops.append(("depol2", (a, b), (float(rng.uniform(0, 0.9)),)))
    got, ref, _ = run_both(vqd_host, n, ops, seed=1, tile_bits=tile_bits, min_contig_bits=3)
    assert_close(got, ref)


def test_c2_grid_small(vqd_host):
    ops = c2_grid_circuit(rows=2, cols=3, n_gates=120)
    got, ref, info = run_both(vqd_host, 6, ops, seed=2, tile_bits=8)
    assert_close(got, ref)
    assert info["n_passes"] < len(ops)


def test_c3_all_to_all_small(vqd_host):
    ops = c3_all_to_all_circuit(n=6, n_gates=60)
    got, ref, _ = run_both(vqd_host, 6, ops, seed=3, tile_bits=8)
    assert_close(got, ref)


def test_named_channels_and_gates(vqd_host):
    n = 4
    ops = [("h", (0,), ()), ("x", (1,), ()), ("y", (2,), ()), ("z", (3,), ()),
           ("su2", (1,), (0.3, -1.2, 0.7, 0.1)), ("cphase", (2, 0), (0.4,)),
           ("xx", (3, 1), (0.9,)), ("gamp", (2,), (0.8, 0.3)), ("bitflip2", (0, 3), (0.2,)),
           ("bitflip1", (1,), (0.1,)), ("amp", (0,), (0.3,)), ("depol1", (3,), (0.2,)),
           ("amp_t1", (2,), (0.5, 20.0)), ("deph_t2", (1,), (0.5, 10.0)), ("deph2", (3, 0), (0.3,))]
    for tb in (4, 8, 12):
        got, ref, _ = run_both(vqd_host, n, ops, seed=4, tile_bits=tb, min_contig_bits=0)
        assert_close(got, ref)


def test_many_runtime_diagonals_fit_lds(vqd_host):
    """A long stream of diagonal ops on qubits outside the register slots (the
    static ZZ coupling and read-out of a device preset) needs more table
    entries than one pass can stage: the planner splits the pass so that the
    tables and the tile fit the 160 KiB of LDS, and the result is unchanged."""
    from tests.test_presets import sc_gates
    n = 6
    dev, _ = vqd_host.Device.preset("superconducting")
    ops = dev.insert_noise(sc_gates(n, 150, 21)) + dev.readout_noise(list(range(n)), 0)
    got, ref, info = run_both(vqd_host, n, ops, seed=3)
    assert_close(got, ref, 1e-11)
    prog = vqd_host.Program(n, ops)
    prog.plan(vqd_host.plan_opts())
    plan = emu.parse(prog.export())
    for p in plan["passes"]:
        L = int(p["L"])
        assert (16 << L) + 16 * int(p["rt_count"]) + 1024 <= 160 * 1024
    assert len(plan["passes"]) > 1


def hermitian_state(n, seed):
    R = start_state(n, seed)
    return (R + R.conj().T) / 2


def run_herm(vqd, n, ops, seed=0, **opts):
    R0 = hermitian_state(n, seed)
    dm = OracleDM(n)
    dm.set(R0)
    emulate(n, ops, dm)
    ref = dm.to_vectorised()
    prog = vqd.Program(n, ops)
    prog.plan(vqd.plan_opts(hermitian=True, **opts))
    plan = emu.parse(prog.export())
    got = emu.run(plan, np.ascontiguousarray(R0.T).reshape(-1))
    return got, ref, prog.info(), plan


@pytest.mark.parametrize("n", [2, 3, 4, 6, 7, 9])
def test_hermitian_mode_circuits(vqd_host, n):
    """Hermitian mode: half the tiles computed, their conjugate transposes
    written to the mirrored tiles; the result equals the oracle's."""
    ops = c1_line_circuit(n=n, n_gates=60) if n < 7 else c2_grid_circuit(rows=1, cols=n, n_gates=80)
    got, ref, info, plan = run_herm(vqd_host, n, ops, seed=n)
    assert info["hermitian"] == 1
    assert_close(got, ref)
    last = len(plan["passes"]) - 1
    for k, P in enumerate(plan["passes"]):
        flags = int(P["herm"])
        assert flags & emu.HERM_PASS and int(P["L"]) % 2 == 0
        # only the computed half is stored between passes; the last restores all
        assert bool(flags & emu.HERM_HALF_IN) == (k > 0)
        assert bool(flags & emu.HERM_MIRROR) == (k == last)


@pytest.mark.parametrize("tile_bits", [8, 10, 12, 13])
def test_hermitian_mode_tile_sizes(vqd_host, tile_bits):
    n = 8
    ops = c3_all_to_all_circuit(n=n, n_gates=60)
    got, ref, info, plan = run_herm(vqd_host, n, ops, seed=1, tile_bits=tile_bits)
    assert_close(got, ref)
    L = min(tile_bits & ~1, 2 * n)
    m = n - L // 2
    assert abs(info["tile_fraction"] - (2 ** m + 1) / 2 ** (m + 1)) <= 1e-15
    # qubits 0..hc-1 are in every tile (hc = 3 unless the widest gate, here
    # two qubits, would not fit beside them); the first and last phases put
    # their row and column bits on the lowest thread bits (coalesced loads,
    # stores and mirrored stores)
    hc = min(3, L // 2 - 2)
    io = list(range(hc)) + [n + q for q in range(hc)]
    for P in plan["passes"]:
        tiles = set(range(2 * n)) - set(int(g) for g in P["group_gpos"][:int(P["ngb"])])
        assert set(io) <= tiles
        for ph in (int(P["pb"]), int(P["pe"]) - 1):
            assert [int(g) for g in plan["phases"][ph]["thr_gpos"][:2 * hc]] == io


def test_hermitian_mode_named_channels_and_wide_gates(vqd_host):
    n = 6
    ops = random_matrix_ops(n, 8, seed=5, max_k=min(4, n), kraus=False)
    ops += [("depol1", (0,), (0.2,)), ("depol2", (1, 3), (0.3,)), ("amp", (2,), (0.4,)),
            ("gamp", (4,), (0.6, 0.3)), ("zz", (5, 0), (0.05,)), ("cz", (1, 4), ()), ("deph2", (2, 5), (0.1,))]
    ops += random_matrix_ops(n, 20, seed=6, max_k=2)
    got, ref, info, _ = run_herm(vqd_host, n, ops, seed=2)
    assert info["hermitian"] == 1
    assert_close(got, ref)


def test_hermitian_mode_refused_for_a_map_that_breaks_hermiticity(vqd_host):
    """An op with S[mu(a)][mu(b)] != conj(S[a][b]) (here rho -> A rho B^dagger
    with A != B) makes the planner fall back to computing every tile."""
    n = 4
    rng = np.random.default_rng(3)
    A = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    B = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    S = np.kron(np.conj(B), A)
    ops = c1_line_circuit(n=n, n_gates=20) + [("superop", (1,), (S,))]
    prog = vqd_host.Program(n, ops)
    prog.plan(vqd_host.plan_opts(hermitian=True))
    assert prog.info()["hermitian"] == 0
    assert prog.info()["tile_fraction"] == 1.0


def _kinds(vqd, n, ops, **opts):
    prog = vqd.Program(n, ops)
    prog.plan(vqd.plan_opts(**opts))
    plan = emu.parse(prog.export())
    return [int(o["kind"]) for o in plan["ops"]], prog.info()


def test_one_qubit_maps_in_pauli_transfer_form(vqd_host):
    """Trace-preserving one-qubit maps that keep Hermitian blocks Hermitian
    are applied through their real Pauli transfer matrix (kernel op kind 5).
    A trace-decreasing M rho M^dagger and a map rho -> A rho B^dagger
    (A != B, complex transfer matrix) stay dense matrices (kind 1).  Each
    result matches the oracle (the last one a direct product here)."""
    n = 3
    rng = np.random.default_rng(11)
    su2 = [("su2", (q,), tuple(float(x) for x in rng.standard_normal(4))) for q in range(n)]
    noisy = su2 + [("amp", (0,), (0.3,)), ("deph1", (1,), (0.2,)), ("depol1", (2,), (0.1,))]
    kinds, _ = _kinds(vqd_host, n, noisy)
    assert kinds and all(k == 5 for k in kinds), kinds
    got, ref, _ = run_both(vqd_host, n, noisy, seed=4)
    assert_close(got, ref)

    M = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) * 0.5
    lossy = [("matrix", (1,), (M,))]
    assert _kinds(vqd_host, n, lossy)[0] == [1]
    got, ref, _ = run_both(vqd_host, n, lossy, seed=5)
    assert_close(got, ref)

    A = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    B = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    skew = [("superop", (2,), (np.kron(np.conj(B), A),))]
    assert _kinds(vqd_host, n, skew)[0] == [1]
    prog = vqd_host.Program(n, skew)
    prog.plan(vqd_host.plan_opts())
    R0 = start_state(n, 6)
    got = emu.run(emu.parse(prog.export()), np.ascontiguousarray(R0.T).reshape(-1))
    # qubit q is index bit q: the full operators with A (B) on qubit 2
    Af = np.kron(A, np.eye(4))
    Bf = np.kron(B, np.eye(4))
    ref = (Af @ R0 @ Bf.conj().T).T.reshape(-1)
    assert_close(got, ref)


@pytest.mark.parametrize("n,tile_bits,contig", [(4, 4, 0), (6, 8, 1), (7, 8, 1), (8, 10, 1), (9, 12, 1), (9, 8, 0)])
def test_relabelled_plans_match_the_oracle(vqd_host, n, tile_bits, contig):
    """relayout: the state between passes is stored under qubit relabellings;
    passes that change it write the other buffer (the emulator starts that
    buffer as NaN, so a read of an amplitude no pass stored shows).  The
    result, in the caller's buffer under the original labelling, equals the
    oracle's; the number of buffer changes is even."""
    ops = c2_grid_circuit(rows=1, cols=n, n_gates=120) if n % 2 else c1_line_circuit(n=n, n_gates=90)
    got, ref, info, plan = run_herm(vqd_host, n, ops, seed=n, tile_bits=tile_bits,
                                    min_contig_bits=contig, relayout=True)
    assert info["hermitian"] == 1
    assert np.isfinite(got).all()
    assert_close(got, ref)
    swaps = [int(P["swap_out"]) for P in plan["passes"]]
    assert sum(swaps) % 2 == 0
    assert info["relabelled"] == (len(plan["passes"]) > 1) and info["layout_changes"] == sum(swaps)


def test_relabelled_grid_circuit_layouts(vqd_host):
    """The 2x5 grid circuit in relabelled Hermitian mode against the oracle.
    Between passes the state is interleaved (a qubit's row and column bits
    are neighbours); the first pass loads and the last stores the vectorised
    layout (the bits of a qubit n apart).  Every pass's group bits come in
    such pairs in both layouts, a pass that keeps its layout stores with the
    group positions it loads, and the lanes of every loading and storing
    phase start with the run of physical positions 0, 1, 2, ... among its
    thread bits."""
    n = 10
    ops = c2_grid_circuit(rows=2, cols=5, n_gates=160)
    got, ref, info, plan = run_herm(vqd_host, n, ops, seed=3, tile_bits=12, min_contig_bits=1, relayout=True)
    assert_close(got, ref)
    passes = plan["passes"]
    assert len(passes) > 2 and sum(int(P["swap_out"]) for P in passes) % 2 == 0
    steps = []        # the layout kind at every boundary: n (vectorised) or 1 (interleaved)
    for k, P in enumerate(passes):
        m = int(P["ngb"]) // 2
        g, o = [int(x) for x in P["group_gpos"][:2 * m]], [int(x) for x in P["out_gpos"][:2 * m]]
        s_in, s_out = {g[m + i] - g[i] for i in range(m)}, {o[m + i] - o[i] for i in range(m)}
        assert len(s_in) == 1 and len(s_out) == 1 and s_in | s_out <= {1, n}
        if k:
            assert s_in == steps[-1]
        steps.append(s_out)
        if k == 0:
            assert s_in == {n}
        if not int(P["swap_out"]):
            assert g == o
    assert steps[-1] == {n} and {1} in steps
    for P in passes:
        nthr = int(P["L"]) - 4
        for ph in (int(P["pb"]), int(P["pe"]) - 1):
            thr = [int(x) for x in plan["phases"][ph]["thr_gpos"][:nthr]]
            r = 0
            while r in thr:
                r += 1
            assert thr[:r] == list(range(r))


def lane_runs(plan, which):
    """Per pass: the run of physical positions 0, 1, 2, ... that lead the
    lanes of its loading (which = 0) or storing (1) phase."""
    out = []
    for P in plan["passes"]:
        ph = int(P["pb"]) if which == 0 else int(P["pe"]) - 1
        thr = [int(x) for x in plan["phases"][ph]["thr_gpos"][:int(P["L"]) - 4]]
        r = 0
        while r < len(thr) and thr[r] == r:
            r += 1
        out.append(r)
    return np.array(out)


def test_relabelling_makes_tiles_contiguous(vqd_host):
    """On the 14-qubit grid circuit's plan, the interleaved layouts put each
    tile's qubits lowest: almost every pass loads whole waves of 64
    consecutive amplitudes (6 or more leading lanes), and half or more store
    runs of 16 or more; the vectorised layout leads with its forced qubits'
    row bits only (runs of 2 to 8).  With relabelled layouts a tile keeps a
    qubit of the previous tile instead of qubit 0, which needs fewer passes
    (136 against 168)."""
    n = 14
    ops = c2_grid_circuit(rows=2, cols=7, n_gates=2000)
    plans = {}
    for rel in (False, True):
        prog = vqd_host.Program(n, ops)
        prog.plan(vqd_host.plan_opts(tile_bits=12, min_contig_bits=1, hermitian=True, relayout=rel))
        plans[rel] = (emu.parse(prog.export()), prog.info())
    assert plans[True][1]["n_passes"] < plans[False][1]["n_passes"]
    # every boundary leads with a qubit both tiles hold, outside the
    # registers of the storing and the loading phase: no 16-byte scatter
    assert lane_runs(plans[True][0], 1).min() >= 2 and lane_runs(plans[True][0], 0)[1:].min() >= 2
    load_rel, store_rel = lane_runs(plans[True][0], 0), lane_runs(plans[True][0], 1)
    load_vec, store_vec = lane_runs(plans[False][0], 0), lane_runs(plans[False][0], 1)
    assert np.mean(load_rel[1:] >= 6) > 0.95
    assert np.mean(store_rel[:-1] >= 4) > 0.5
    assert load_vec[1:].max() <= 3 and store_vec.max() <= 3


def exchange_bank_degrees(plan, lanes=16, groups=16):
    """Per LDS exchange access (a phase's 16 register slots, written at its
    end or read at its start) and per group of `lanes` consecutive lanes: the
    largest number of lanes that hit one of `groups` 16-byte bank groups
    under the kernel's xor swizzle of the tile-local index."""
    def swz(l):
        return l ^ (((l >> 4) ^ (l >> 8)) & 15)
    out = []
    for P in plan["passes"]:
        pb, pe, nthr = int(P["pb"]), int(P["pe"]), int(P["L"]) - 4
        for ph in range(pb, pe):
            uses = (ph != pb) + (ph + 1 < pe)
            if not uses:
                continue
            tl, _, sl, _, _, _ = emu._phase_parts(plan["phases"][ph], nthr)
            tl, sl = tl.astype(np.int64), sl.astype(np.int64)
            for e in range(16):
                bank = swz(tl ^ sl[e]) % groups
                for g in range(0, tl.size, lanes):
                    out += [np.bincount(bank[g:g + lanes], minlength=groups).max()] * uses
    return np.array(out)


@pytest.mark.parametrize("relayout", [False, True])
def test_exchanges_spread_lds_banks(vqd_host, relayout):
    """The planner orders every exchange phase's lanes, and permutes each
    pass's tile-local bit labels, so that the 16 lanes of a 128-bit LDS
    access (and any 8 of them) reach distinct bank groups: on the 14-qubit
    grid circuit's plan nearly every access is conflict-free.  In the
    vectorised layout a register set can hold three tile bits of one residue,
    which leaves a phase's thread bits without it (a few conflicts remain)."""
    prog = vqd_host.Program(14, c2_grid_circuit(rows=2, cols=7, n_gates=2000))
    prog.plan(vqd_host.plan_opts(tile_bits=12, min_contig_bits=1, hermitian=True, relayout=relayout))
    plan = emu.parse(prog.export())
    d16 = exchange_bank_degrees(plan, 16, 16)
    d8 = exchange_bank_degrees(plan, 8, 8)
    bound = 1.02 if relayout else 1.08
    assert d16.mean() <= bound and d8.mean() <= bound, (d16.mean(), d8.mean())
    assert np.mean(d16 == 1) >= (0.98 if relayout else 0.9)
