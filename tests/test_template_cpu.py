"""Parametric templates on the host: a circuit structure planned once with
generic parameters, then given each instance's own coefficients.  The
exported descriptors are run through the CPU emulation of the pass kernel
and compared with the oracle at 1e-10."""
import numpy as np
import pytest

from oracle.emulator import emulate
from tests import _plan_emu
from workloads import c5_ansatz_circuit, c5_draw_samples, c5_params, c5_structure

TOL = 1e-10

# named kinds with (arity, parameter sampler)
KIND_SPECS = {
    "rx": (1, lambda r: [r.uniform(0, 6.3)]), "ry": (1, lambda r: [r.uniform(0, 6.3)]),
    "rz": (1, lambda r: [r.uniform(0, 6.3)]), "h": (1, lambda r: []), "x": (1, lambda r: []),
    "y": (1, lambda r: []), "z": (1, lambda r: []), "su2": (1, lambda r: list(r.standard_normal(4))),
    "cz": (2, lambda r: []), "cphase": (2, lambda r: [r.uniform(0, 6.3)]),
    "xx": (2, lambda r: [r.uniform(0, 6.3)]), "zz": (2, lambda r: [r.uniform(-0.1, 0.1)]),
    "depol1": (1, lambda r: [r.uniform(0, 0.05)]), "depol2": (2, lambda r: [r.uniform(0, 0.05)]),
    "deph1": (1, lambda r: [r.uniform(0, 0.05)]), "deph2": (2, lambda r: [r.uniform(0, 0.05)]),
    "amp": (1, lambda r: [r.uniform(0, 0.05)]), "gamp": (1, lambda r: [r.uniform(0, 1), r.uniform(0, 0.05)]),
    "bitflip1": (1, lambda r: [r.uniform(0, 0.05)]), "bitflip2": (2, lambda r: [r.uniform(0, 0.05)]),
    "amp_t1": (1, lambda r: [r.uniform(0.02, 0.8), r.uniform(20, 200)]),
    "deph_t2": (1, lambda r: [r.uniform(0.02, 0.8), r.uniform(10, 100)]),
}


N_PARAMS = {k: len(spec[1](np.random.default_rng(0))) for k, spec in KIND_SPECS.items()}


def random_structure(n, count, seed):
    rng = np.random.default_rng(seed)
    names = sorted(KIND_SPECS)
    structure = []
    for _ in range(count):
        k = names[int(rng.integers(len(names)))]
        a = KIND_SPECS[k][0]
        structure.append((k, tuple(int(x) for x in rng.choice(n, a, replace=False))))
    return structure


def random_params(structure, seed):
    rng = np.random.default_rng(seed)
    P = np.zeros((len(structure), 4))
    for i, (k, _) in enumerate(structure):
        v = KIND_SPECS[k][1](rng)
        P[i, :len(v)] = v
    return P


def as_ops(structure, P):
    return [(k, q, tuple(float(x) for x in P[i, :N_PARAMS[k]])) for i, (k, q) in enumerate(structure)]


def run_template(vqd, n, structure, P, opts=None):
    plan = _plan_emu.parse(vqd.template_export(n, structure, P, opts))
    rho0 = np.zeros(4 ** n, dtype=complex)
    rho0[0] = 1
    return _plan_emu.run(plan, rho0)


def test_c5_structure_matches_ansatz_generator():
    dev, ang = c5_draw_samples(3, seed=11)
    st = c5_structure()
    P = c5_params(st, dev, ang)
    for s in range(3):
        ref = c5_ansatz_circuit(dev[s], ang[s])
        got = [(k, q, tuple(P[s, i, :len(sl)])) for i, (k, q, sl) in enumerate(st)]
        assert dev[s, 6] != 0.0
        assert got == ref


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_structure_instances_match_oracle(vqd_host, seed):
    n = 5
    structure = random_structure(n, 60, seed=100 + seed)
    for inst in range(2):
        P = random_params(structure, seed=1000 * seed + inst)
        ops = as_ops(structure, P)
        got = run_template(vqd_host, n, structure, P, vqd_host.plan_opts(tile_bits=8, min_contig_bits=2))
        ref = emulate(n, ops).to_vectorised()
        assert np.abs(got - ref).max() <= TOL, (seed, inst)


def test_template_keeps_identity_parameters(vqd_host):
    """Parameters that make ops the identity (p = 0, angle 0, alpha 0) keep
    the slots planned for generic values and still give the oracle's state."""
    n = 4
    structure = [("ry", (0,)), ("depol1", (0,)), ("cz", (0, 1)), ("zz", (1, 2)), ("rx", (2,)),
                 ("amp_t1", (3,)), ("deph2", (2, 3)), ("rz", (1,))]
    P = np.zeros((len(structure), 4))
    P[0, 0] = 0.4
    P[5, :2] = (0.1, 50.0)
    ops = as_ops(structure, P)
    got = run_template(vqd_host, n, structure, P, vqd_host.plan_opts(tile_bits=6, min_contig_bits=2))
    assert np.abs(got - emulate(n, ops).to_vectorised()).max() <= TOL


def test_c5_small_instances_match_oracle(vqd_host):
    n, layers = 6, 2
    st = c5_structure(n=n, layers=layers)
    dev, ang = c5_draw_samples(3, seed=5, n_angles=4 * layers)
    P = c5_params(st, dev, ang)
    structure = [(k, q) for k, q, _ in st]
    for s in range(3):
        got = run_template(vqd_host, n, structure, P[s], vqd_host.plan_opts(tile_bits=12, min_contig_bits=3))
        ref = emulate(n, c5_ansatz_circuit(dev[s], ang[s], n=n, layers=layers)).to_vectorised()
        assert np.abs(got - ref).max() <= TOL, s


def test_c5_full_instance_matches_oracle(vqd_host):
    """The 10-qubit, 4-layer ansatz in the batched tile configuration."""
    st = c5_structure()
    dev, ang = c5_draw_samples(1, seed=9)
    P = c5_params(st, dev, ang)[0]
    structure = [(k, q) for k, q, _ in st]
    got = run_template(vqd_host, 10, structure, P, vqd_host.plan_opts(tile_bits=12, min_contig_bits=3,
                                                                      pad_coalesce=False))
    ref = emulate(10, c5_ansatz_circuit(dev[0], ang[0])).to_vectorised()
    assert np.abs(got - ref).max() <= TOL


def test_template_plan_equals_program_plan_for_generic_parameters(vqd_host):
    """With generic parameters the structure planned from the template's
    canonical values is the one the ordinary planner picks for the instance,
    and the recomputed coefficients are the same numbers."""
    n = 6
    st = c5_structure(n=n, layers=2)
    dev, ang = c5_draw_samples(1, seed=3, n_angles=8)
    P = c5_params(st, dev, ang)[0]
    structure = [(k, q) for k, q, _ in st]
    opts = vqd_host.plan_opts(tile_bits=10, min_contig_bits=3)
    a = _plan_emu.parse(vqd_host.template_export(n, structure, P, opts))
    prog = vqd_host.Program(n, c5_ansatz_circuit(dev[0], ang[0], n=n, layers=2)).plan(opts)
    b = _plan_emu.parse(prog.export())
    for key in ("passes", "phases", "ops"):
        assert a[key].tobytes() == b[key].tobytes(), key
    assert np.abs(a["mats"] - b["mats"]).max() <= 1e-14


def test_template_rejects_bad_input(vqd_host):
    with pytest.raises(vqd_host.VQDError):
        vqd_host.template_export(3, [("cz", (0, 0))])
    with pytest.raises(vqd_host.VQDError):
        vqd_host.template_export(3, [("rx", (3,))])
    P = np.zeros((1, 4))
    P[0, 0] = np.nan
    with pytest.raises(vqd_host.VQDError):
        vqd_host.template_export(3, [("rx", (0,))], P)


@pytest.mark.parametrize("seed", [3, 4])
def test_hermitian_template_instances_match_oracle(vqd_host, seed):
    """Templates in Hermitian mode (the batched kernel's default plan): the
    structure planned once, each instance's coefficients filled in, half the
    tiles computed and the rest restored as conjugate transposes."""
    n = 6
    structure = random_structure(n, 50, seed=200 + seed)
    for inst in range(2):
        P = random_params(structure, seed=2000 * seed + inst)
        got = run_template(vqd_host, n, structure, P,
                           vqd_host.plan_opts(tile_bits=8, min_contig_bits=1, hermitian=True))
        ref = emulate(n, as_ops(structure, P)).to_vectorised()
        assert np.abs(got - ref).max() <= TOL


def test_batch_default_plan_is_hermitian(vqd_host):
    b = vqd_host.Batch()
    b.add(9, [("h", (0,), ())])
    o = b.plan_opts(9)
    assert o["hermitian"] == 1 and o["min_contig_bits"] == 1
