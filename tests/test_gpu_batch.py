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


def test_template_instances_match_oracle(gpu_lib):
    """Parametric templates (one planned structure, per-instance parameters)
    mixed with ordinary instances in one batch; the instance indices follow
    the order of addition."""
    from workloads import c5_ansatz_circuit, c5_draw_samples, c5_params, c5_structure
    say("template batch")
    insts = mixed_instances(seed=3)[:4]
    b = gpu_lib.Batch()
    b.add(*insts[0])
    st6 = c5_structure(n=6, layers=2)
    dev6, ang6 = c5_draw_samples(5, seed=21, n_angles=8)
    t6 = b.add_template(6, [(k, q) for k, q, _ in st6])
    idx6 = b.add_instances(t6, c5_params(st6, dev6, ang6)[:3])
    b.add(*insts[1])
    st10 = c5_structure()
    dev10, ang10 = c5_draw_samples(3, seed=22)
    t10 = b.add_template(10, [(k, q) for k, q, _ in st10])
    idx10 = b.add_instances(t10, c5_params(st10, dev10, ang10))
    idx6b = b.add_instances(t6, c5_params(st6, dev6, ang6)[3:])
    assert list(idx6) == [1, 2, 3] and list(idx10) == [5, 6, 7] and list(idx6b) == [8, 9]
    b.compile()
    assert b.info()["n_instances"] == 10
    b.run()
    for i, (n, ops) in zip((0, 4), insts[:2]):
        ref = emulate(n, ops)
        assert np.abs(b.state(i) - ref.to_vectorised()).max() <= TOL
    for j, i in enumerate(list(idx6) + list(idx6b)):
        ref = emulate(6, c5_ansatz_circuit(dev6[j], ang6[j], n=6, layers=2))
        assert np.abs(b.state(i) - ref.to_vectorised()).max() <= TOL, i
        assert np.abs(b.expec_z(i) - ref.expec_z()).max() <= TOL, i
    for j, i in enumerate(idx10):
        ref = emulate(10, c5_ansatz_circuit(dev10[j], ang10[j]))
        assert np.abs(b.state(i) - ref.to_vectorised()).max() <= TOL, i
        assert np.abs(b.expec_z(i) - ref.expec_z()).max() <= TOL, i


def test_template_only_batch_graph_and_autotune(gpu_lib):
    """A batch made only of template instances: autotuned (on a sample of
    them), graph-replayed, and checked against the oracle on a sample."""
    import torch
    from workloads import c5_ansatz_circuit, c5_draw_samples, c5_params, c5_structure
    say("template-only batch")
    st = c5_structure()
    dev, ang = c5_draw_samples(256, seed=23)
    b = gpu_lib.Batch()
    t = b.add_template(10, [(k, q) for k, q, _ in st])
    idx = b.add_instances(t, c5_params(st, dev, ang))
    b.compile()
    with tempfile.TemporaryDirectory() as d:
        b.autotune(os.path.join(d, "tune.json"), max_per_n=16)
        assert ":n10" in open(os.path.join(d, "tune.json")).read()
    b.compile()
    b.run()
    eager = b.out.clone()
    for rep in range(3):
        b.out.zero_()
        torch.cuda.synchronize()
        b.run(use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(b.out, eager), rep
    for j in (0, 77, 255):
        ref = emulate(10, c5_ansatz_circuit(dev[j], ang[j]))
        assert np.abs(b.expec_z(idx[j]) - ref.expec_z()).max() <= TOL, j


def test_device_preset_streams_in_one_batch(gpu_lib):
    """Noisy streams of the three device presets (silicon: off-resonant
    drives, exchange crosstalk, serial; trapped ions; superconducting), twelve
    instances in one persistent launch, each against the oracle."""
    from tests.test_device_oracle import random_gates
    from tests.test_presets import sc_gates, si_gates
    insts = []
    for i in range(12):
        name = ("silicon", "trapped_ion", "superconducting")[i % 3]
        dev, _ = gpu_lib.Device.preset(name)
        n = dev.n
        gates = (si_gates(n, 30, 400 + i) if name == "silicon" else
                 random_gates(n, 30, 400 + i) if name == "trapped_ion" else sc_gates(n, 30, 400 + i))
        insts.append((n, dev.insert_noise(gates)))
    say("preset batch: %d instances, %d ops" % (len(insts), sum(len(o) for _, o in insts)))
    refs = [emulate(n, ops) for n, ops in insts]
    b = gpu_lib.Batch()
    for n, ops in insts:
        b.add(n, ops)
    b.compile()
    b.run()
    check_batch(gpu_lib, b, insts, refs)


def test_batch_reports_the_work_of_its_plans(gpu_lib, mixed):
    """vqd_batch_info's executed FMAs and algorithmic bytes equal the sums,
    over the instances, of each instance's own plan (planned on the host with
    the batch's options for its qubit count)."""
    insts, _ = mixed
    b = gpu_lib.Batch()
    for n, ops in insts:
        b.add(n, ops)
    b.compile()
    info = b.info()
    fma = byts = 0.0
    for n, ops in insts:
        o = b.plan_opts(n)
        p = gpu_lib.Program(n, ops)
        p.plan(gpu_lib.plan_opts(tile_bits=o["tile_bits"], min_contig_bits=o["min_contig_bits"],
                                 max_ops_per_pass=o["max_ops_per_pass"], fuse_blocks=bool(o["fuse_blocks"]),
                                 pad_coalesce=bool(o["pad_coalesce"]), hermitian=bool(o["hermitian"])))
        pi = p.info()
        amps, f = 4.0 ** n, pi["tile_fraction"]
        fma += pi["fma_per_amp"] * f * amps
        byts += 16 * amps + 32 * f * amps * pi["n_passes"] + (16 * (1 - f) * amps if pi["hermitian"] else 0) \
            + 16 * 2.0 ** n
        p.close()
    say("batch work", info["fp64_fma"], fma, info["pass_bytes"], byts)
    assert abs(info["fp64_fma"] - fma) <= 1e-12 * fma
    assert abs(info["pass_bytes"] - byts) <= 1e-12 * byts
    assert info["total_passes"] > 0
