"""Batched runs (one persistent launch for many density matrices) against the
oracle, instance by instance, at 1e-10."""
import os
import sys
import tempfile

import numpy as np
import pytest

from oracle.emulator import emulate
from workloads import c1_line_circuit, c4_batch_instances, random_matrix_ops

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_instances(seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i, n in enumerate([2, 3, 4, 5, 6, 7, 8, 3, 6, 7, 2, 5]):
        if i % 3 == 0:
            ops = random_matrix_ops(n, 25, seed=100 + i, max_k=2)
        else:
            ops = c1_line_circuit(n=n, n_gates=int(rng.integers(20, 60)), seed=200 + i)
        out.append((n, ops))
    return out


def check_batch(vqd, batch, insts, refs):
    for i, (n, ops) in enumerate(insts):
        ref = refs[i]
        got = batch.state(i)
        err = np.abs(got - ref.to_vectorised()).max()
        assert err <= TOL, (i, n, err)
        assert np.abs(batch.expec_z(i) - ref.expec_z()).max() <= TOL


@pytest.fixture(scope="module")
def mixed():
    insts = mixed_instances()
    refs = [emulate(n, ops) for n, ops in insts]
    return insts, refs


@pytest.mark.parametrize("tile_bits", [None, 8, 6])
def test_mixed_batch_matches_oracle(gpu_lib, mixed, tile_bits):
    say("mixed batch tile_bits=%s" % tile_bits)
    insts, refs = mixed
    b = gpu_lib.Batch()
    for n, ops in insts:
        b.add(n, ops)
    if tile_bits is not None:
        for n in set(n for n, _ in insts):
            b.set_opts(n, gpu_lib.plan_opts(tile_bits=min(tile_bits, 2 * n), min_contig_bits=2))
    b.compile()
    b.run()
    check_batch(gpu_lib, b, insts, refs)


def test_batch_graph_replays(gpu_lib, mixed):
    """The captured launch (queue reset + persistent kernel) is replayed
    several times with eager work and synchronisation in between; every replay
    must give the eager result."""
    import torch
    say("graph replays")
    insts, refs = mixed
    b = gpu_lib.Batch()
    for n, ops in insts:
        b.add(n, ops)
    b.compile()
    b.run()
    eager = b.out.clone()
    for rep in range(4):
        b.arena.zero_()
        b.out.zero_()
        torch.cuda.synchronize()
        b.run(use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(b.out, eager), rep
        check_batch(gpu_lib, b, insts, refs)
        b.run()                                   # eager run between replays
        torch.cuda.synchronize()
        assert torch.equal(b.out, eager)


def test_autotuner_writes_cache_and_keeps_results(gpu_lib, mixed):
    say("autotune")
    insts, refs = mixed
    b = gpu_lib.Batch()
    for n, ops in insts:
        b.add(n, ops)
    b.compile()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        b.autotune(path, max_per_n=4)
        text = open(path).read()
        assert ":n7" in text and ":n8" in text
        b.compile()
        b.run()
        check_batch(gpu_lib, b, insts, refs)
        # second tuner call reads the cache instead of timing
        b2 = gpu_lib.Batch()
        for n, ops in insts:
            b2.add(n, ops)
        b2.compile()
        b2.autotune(path, max_per_n=4)
        for n in (7, 8):
            assert b2.plan_opts(n)["tile_bits"] == b.plan_opts(n)["tile_bits"]


def test_full_batch_workload(gpu_lib):
    """The 4096-instance workload (3..10 qubits, 100-400 gates each, own noise
    parameters): sampled instances against the oracle (up to 8 qubits) and
    against the single-density-matrix path (9 and 10 qubits)."""
    say("full batch: generating")
    insts = c4_batch_instances(4096)
    b = gpu_lib.Batch()
    for x in insts:
        b.add(x["n"], x["ops"])
    say("compiling")
    b.compile()
    say("running", b.info())
    b.run()
    out = b.out.cpu().numpy()
    assert np.all(np.isfinite(out)) and np.all(np.abs(out) <= 1 + 1e-12)
    rng = np.random.default_rng(5)
    small = [i for i, x in enumerate(insts) if x["n"] <= 8]
    for i in rng.choice(small, 24, replace=False):
        x = insts[i]
        ref = emulate(x["n"], x["ops"])
        assert np.abs(b.state(int(i)) - ref.to_vectorised()).max() <= TOL
        assert np.abs(b.expec_z(int(i)) - ref.expec_z()).max() <= TOL
    big = [i for i, x in enumerate(insts) if x["n"] >= 9]
    for i in rng.choice(big, 6, replace=False):
        x = insts[int(i)]
        dm = gpu_lib.DensityMatrix(x["n"])
        gpu_lib.Program(x["n"], x["ops"]).compile().run(dm)
        assert np.abs(b.state(int(i)) - dm.to_numpy()).max() <= TOL
        assert np.abs(b.expec_z(int(i)) - dm.expec_z()).max() <= TOL
