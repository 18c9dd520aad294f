"""Device-output read-outs (vqd_calc_*_dev) and a whole step captured in one
HIP graph: init, a planned program and every read-out.

The device forms run the same kernels in the same order as the synchronous
read-outs, so their values must be bit-identical to those; both are checked
against the CPU oracle at 1e-10.  The graph is replayed several times with
eager work of the program's own (init to another state, synchronisations) in
between, and every replay is compared with the eager results.
"""
import sys

import numpy as np
import pytest

from oracle.emulator import emulate, readouts
from workloads import c1_line_circuit, c2_grid_circuit

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def all_pairs(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def dev_outputs(torch, n, npairs):
    f = dict(dtype=torch.float64, device="cuda")
    return {"trace": torch.full((2,), np.nan, **f), "purity": torch.full((1,), np.nan, **f),
            "probs": torch.full((1 << n,), np.nan, **f), "z": torch.full((n,), np.nan, **f),
            "zz": torch.full((max(npairs, 1),), np.nan, **f), "pauli": torch.full((2,), np.nan, **f)}


def enqueue_readouts(dm, out, pairs_dev, codes):
    dm.trace_dev(out["trace"])
    dm.purity_dev(out["purity"])
    dm.probs_dev(out["probs"])
    dm.expec_z_dev(out["z"])
    dm.expec_zz_dev(pairs_dev, out["zz"])
    dm.expec_pauli_dev(codes, out["pauli"])


def host(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


@pytest.mark.parametrize("n,hermitian", [(3, False), (6, False), (8, True), (10, True)])
def test_dev_readouts_match_sync_and_oracle(gpu_lib, n, hermitian):
    import torch
    say("device read-outs n=%d hermitian=%s" % (n, hermitian))
    ops = c1_line_circuit(n=n, n_gates=80)
    opts = gpu_lib.plan_opts(hermitian=True, tile_bits=min(12, 2 * n) & ~1, min_contig_bits=1) if hermitian \
        else gpu_lib.plan_opts()
    prog = gpu_lib.Program(n, ops).compile(opts)
    dm = gpu_lib.DensityMatrix(n)
    prog.run(dm)
    pairs = all_pairs(n)
    pairs_dev = torch.as_tensor(np.asarray(pairs, dtype=np.int32).reshape(-1, 2), device="cuda")
    codes = np.array([(1 + q) % 4 for q in range(n)], dtype=np.uint8)
    out = dev_outputs(torch, n, len(pairs))
    enqueue_readouts(dm, out, pairs_dev, codes)
    torch.cuda.synchronize()
    got = host(out)
    # bit-identical to the synchronous calls (same kernels, same order)
    tr = dm.trace()
    assert got["trace"][0] == tr.real and got["trace"][1] == tr.imag
    assert got["purity"][0] == dm.purity()
    assert np.array_equal(got["probs"], dm.probs())
    assert np.array_equal(got["z"], dm.expec_z())
    assert np.array_equal(got["zz"][:len(pairs)], dm.expec_zz(pairs))
    pa = dm.expec_pauli(codes)
    assert got["pauli"][0] == pa.real and got["pauli"][1] == pa.imag
    # and the oracle
    ref = emulate(n, ops)
    r = readouts(ref, pairs=pairs)
    assert abs(got["trace"][0] - r["trace"].real) <= TOL and abs(got["trace"][1] - r["trace"].imag) <= TOL
    assert abs(got["purity"][0] - r["purity"]) <= TOL
    assert np.abs(got["probs"] - r["probs"]).max() <= TOL
    assert np.abs(got["z"] - r["expec_z"]).max() <= TOL
    assert np.abs(got["zz"][:len(pairs)] - r["expec_zz"]).max() <= TOL
    want = ref.expec_pauli(codes)
    assert abs(got["pauli"][0] - want.real) <= TOL and abs(got["pauli"][1] - want.imag) <= TOL


def test_dev_readout_argument_errors(gpu_lib):
    import torch
    dm = gpu_lib.DensityMatrix(3)
    bad = torch.zeros(2, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        dm.trace_dev(bad)
    with pytest.raises(gpu_lib.VQDError):
        dm.expec_pauli_dev(np.array([0, 4, 0], dtype=np.uint8), torch.zeros(2, dtype=torch.float64,
                                                                             device="cuda"))


@pytest.mark.parametrize("n", [7, 12])
def test_whole_step_in_one_graph(gpu_lib, n):
    """init + program (Hermitian plan at 12 qubits) + read-outs captured on
    the handle's stream; each replay equals the eager step bit for bit and
    the oracle within 1e-10."""
    import torch
    say("graph capture n=%d" % n)
    if n == 12:
        ops = c2_grid_circuit(rows=2, cols=6, n_gates=120)
        opts = gpu_lib.plan_opts(hermitian=True, tile_bits=12, min_contig_bits=1)
    else:
        ops = c1_line_circuit(n=n, n_gates=120)
        opts = gpu_lib.plan_opts()
    s = torch.cuda.Stream()
    pairs = all_pairs(n)
    pairs_dev = torch.as_tensor(np.asarray(pairs, dtype=np.int32).reshape(-1, 2), device="cuda")
    codes = np.array([3 if q % 3 == 0 else 1 if q % 3 == 1 else 0 for q in range(n)], dtype=np.uint8)
    with torch.cuda.stream(s):
        dm = gpu_lib.DensityMatrix(n, stream=s)
        prog = gpu_lib.Program(n, ops).compile(opts)
        out = dev_outputs(torch, n, len(pairs))
        # eager step (also sets the kernels' launch attributes before capture)
        dm.init_zero()
        prog.run(dm)
        enqueue_readouts(dm, out, pairs_dev, codes)
    s.synchronize()
    eager = host(out)
    eager_state = dm.to_numpy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        dm.init_zero()
        prog.run(dm)
        enqueue_readouts(dm, out, pairs_dev, codes)
    ref = emulate(n, ops)
    r = readouts(ref, pairs=pairs)
    for rep in range(4):
        # eager work between replays: another initial state, cleared outputs
        with torch.cuda.stream(s):
            dm.init_basis(rep + 1)
            for v in out.values():
                v.fill_(np.nan)
        s.synchronize()
        g.replay()
        s.synchronize()
        got = host(out)
        for k in eager:
            assert np.array_equal(got[k], eager[k]), (rep, k)
        assert np.array_equal(dm.to_numpy(), eager_state), rep
        assert np.abs(got["z"] - r["expec_z"]).max() <= TOL
        assert abs(got["purity"][0] - r["purity"]) <= TOL
        assert np.abs(got["probs"] - r["probs"]).max() <= TOL
        assert np.abs(got["zz"][:len(pairs)] - r["expec_zz"]).max() <= TOL
        assert abs(got["trace"][0] - 1.0) <= TOL
        want = ref.expec_pauli(codes)
        assert abs(got["pauli"][0] - want.real) <= TOL and abs(got["pauli"][1] - want.imag) <= TOL
    say("graph replays ok")
