#!/usr/bin/env python3
"""Benchmark of the density-matrix emulation hot path on one MI355X.

A step is one whole noisy circuit on the 14-qubit density matrix (4^14
complex128 amplitudes, 4.29 GB): init |0..0><0..0|, every gate and channel of
the seeded 2x7-grid circuit (2000 SU(2)/CZ gates, 9378 density-matrix ops in
all, including depolarising, T1/T2 and ZZ-crosstalk ops), then the read-outs
<Z_i> and purity.  The op program is planned once (outside the timed region)
into fused HBM passes.

Prints one JSON line (see the fields below).  `value` is density-matrix ops
per second (gates and channels); gates-only throughput is reported beside it.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DM gate-ops/s & HBM GB/s at 14q; surrogate vs emulator evals/s @ |ΔZ|<1e-2"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
N_QUBITS = 14
# planner options of the timed configuration (the GPU parity tests use the same)
# Hermitian mode (the state is a density matrix and every op is a Kraus map or
# a unitary): each pass computes the tiles whose row group index is at most
# the column one, 12-bit tiles of whole qubits with qubit 0 in every tile
PLAN_OPTS = dict(tile_bits=12, min_contig_bits=1, max_ops_per_pass=0, fuse_blocks=True, pad_coalesce=True,
                 hermitian=True, relayout=True)


def pass_bytes(info, amps):
    """HBM bytes of all passes of one run: every computed amplitude is read
    and written once per pass (16 B each way); in Hermitian mode only the
    fraction f of the amplitudes is computed and stored between passes, and
    the last pass also writes the other 1 - f (the mirror images)."""
    f = info["tile_fraction"]
    return amps * (32.0 * f * info["n_passes"] + (16.0 * (1.0 - f) if info["hermitian"] else 0.0))


def executed_flops(info, amps):
    """FP64 flops the passes execute: 2 per planned FMA per computed amplitude."""
    return 2.0 * info["fma_per_amp"] * info["tile_fraction"] * amps
# HBM traffic of the pass kernel measured with rocprofv3 counters (FETCH_SIZE,
# WRITE_SIZE) on this workload; valid only for the kernel source it was taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_grid14_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2306_07342_amd", "csrc", f)
                  for f in ("kernels.hip", "dev_common.h", "planner.cpp")]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per pass-kernel launch from the committed counter summary, or
    None when it is missing or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload():
    from workloads import c2_grid_circuit
    ops = c2_grid_circuit(rows=2, cols=7, n_gates=2000)
    n_gates = sum(1 for k, _, _ in ops if k in ("su2", "cz"))
    return ops, n_gates


def cpu_baseline(ops, n, sample_every):
    """The oracle (as it is) on a bounded sample of the same workload: every
    `sample_every`-th op of the circuit applied to a 14-qubit state."""
    from oracle.core import OracleDM
    from oracle.emulator import emulate
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sample = ops[::sample_every]
    dm = OracleDM(n)
    t0 = time.perf_counter()
    emulate(n, sample, dm)
    dt = time.perf_counter() - t0
    return {"value": len(sample) / dt, "unit": "DM ops/s", "cores": threads, "kind": "oracle",
            "sample": "%d ops (every %d-th op of the 14-qubit grid circuit) on a 14-qubit state, %.1f s"
                      % (len(sample), sample_every, dt)}


BATCH_TUNE_FILE = os.path.join(ROOT, "paper_2306_07342_amd", "tune", "batch_tiles.json")
C5_TUNE_FILE = os.path.join(ROOT, "paper_2306_07342_amd", "tune", "c5_template_tiles.json")


def batched_leg(vqd, torch, steps):
    """4096 independent 3..10-qubit noisy line circuits (own noise parameters)
    in one persistent, graph-captured launch; its FP64 and HBM fractions from
    the work the instances' plans execute; against the single-density-matrix
    path over a random subset of 512 of them, looped inside one HIP graph
    (init, program and a device-output read-out per circuit, no host
    synchronisation in between) and, for context, looped eagerly."""
    import random
    from workloads import c4_batch_instances
    t0 = time.perf_counter()
    insts = c4_batch_instances(4096)
    n_ops = sum(len(x["ops"]) for x in insts)

    def make(sel):
        b = vqd.Batch()
        for i in sel:
            b.add(insts[i]["n"], insts[i]["ops"])
        return b

    b = make(range(len(insts)))
    b.compile()
    tuned = os.path.exists(BATCH_TUNE_FILE)
    b.autotune(BATCH_TUNE_FILE if tuned else os.path.join("/tmp", "vqd_batch_tiles.json"), max_per_n=32)
    b.compile()
    info = b.info()
    log("batched: setup %.1f s, %s" % (time.perf_counter() - t0, info))
    stream = torch.cuda.current_stream()

    def timed(fn, reps, st=None):
        st = st or stream
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    t_batch = timed(lambda: b.run(use_graph=True), max(1, steps))
    tf = 2.0 * info["fp64_fma"] / t_batch / 1e12
    gbs = info["pass_bytes"] / t_batch / 1e9
    # the same circuits, one single-state program each: 512 of them
    sel = random.Random(7).sample(range(len(insts)), 512)
    s = torch.cuda.Stream()
    zs = torch.empty(sum(insts[i]["n"] for i in sel), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        progs = [(insts[i]["n"], vqd.Program(insts[i]["n"], insts[i]["ops"]).compile()) for i in sel]
        dms = {}
        for n, _ in progs:
            if n not in dms:
                dms[n] = vqd.DensityMatrix(n, stream=s)

    def loop():
        off = 0
        for n, p in progs:
            dm = dms[n]
            dm.init_zero()
            p.run(dm)
            dm.expec_z_dev(zs[off:off + n])
            off += n

    with torch.cuda.stream(s):
        t_loop_eager = timed(loop, 1, s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            loop()
        t_loop_graph = timed(g.replay, max(1, steps), s)
    sub = make(sel)
    sub.compile()
    t_sub = timed(lambda: sub.run(use_graph=True), max(1, steps))
    return {"metric": "batched noisy circuits per second (4096 density matrices, 3-10 qubits)",
            "circuits_per_s": round(len(insts) / t_batch, 1),
            "dm_ops_per_s": round(n_ops / t_batch, 1),
            "ms_per_batch": round(t_batch * 1e3, 3),
            "dm_ops": n_ops,
            "roofline": {"alu": {"achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(tf / FP64_PEAK_TFLOPS, 4)},
                         "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(gbs / HBM_PEAK_GBS, 4)},
                         "work": "executed FMAs and algorithmic bytes of the instances' plans, per run"},
            "subset512_batched_ms": round(t_sub * 1e3, 3),
            "subset512_single_path_in_one_graph_ms": round(t_loop_graph * 1e3, 3),
            "subset512_single_path_eager_ms": round(t_loop_eager * 1e3, 3),
            "speedup_vs_single_path_graph": round(t_loop_graph / t_sub, 2),
            "tiles": "autotuned (%s)" % ("cached" if tuned else "fresh")}


def c3_leg(vqd, torch, steps: int):
    """Context beside the 14-qubit metric: the seeded 16-qubit all-to-all
    circuit (500 XX/Ry/Rz gates with depol2 and dephasing) on a 64 GiB
    density matrix, one warm-up and `steps` timed steps."""
    from workloads import c3_all_to_all_circuit
    n = 16
    ops = c3_all_to_all_circuit(n=n, n_gates=500)
    n_gates = sum(1 for k, _, _ in ops if k in ("xx", "ry", "rz"))
    prog = vqd.Program(n, ops).compile(vqd.plan_opts(**PLAN_OPTS))
    info = prog.info()
    dm = vqd.DensityMatrix(n)
    stream = torch.cuda.current_stream()

    def step():
        dm.init_zero()
        prog.run(dm)
        return dm.expec_z(), dm.purity()

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        z, pur = step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    amps = 4 ** n
    t_pass = e0.elapsed_time(e1) / 1e3 / steps       # includes init and read-outs
    gbs = pass_bytes(info, amps) / t_pass / 1e9
    tf = executed_flops(info, amps) / t_pass / 1e12
    out = {"workload": "16-qubit density matrix (complex128, 4^16 amps, 68.7 GB), all-to-all circuit, "
                       "500 XX/Ry/Rz gates with depol2(1e-2) and deph(1e-3)",
           "dm_ops_per_s": round(len(ops) / wall, 1), "gates_per_s": round(n_gates / wall, 1),
           "ms_per_step": round(wall * 1e3, 2), "dm_ops": len(ops), "passes": info["n_passes"],
           "hermitian_mode": bool(info["hermitian"]),
           "hbm_gbs_of_passes": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "fp64_tflops": round(tf, 2), "alu_frac": round(tf / FP64_PEAK_TFLOPS, 4),
           "check": {"purity": float(pur), "z0": float(z[0])}}
    del dm
    torch.cuda.empty_cache()
    return out


def traj_leg(vqd, torch, n_traj: int, steps: int, oracle_sample: bool):
    """Monte Carlo trajectories of the 12-qubit grid circuit (2x6 grid, 2000
    gates, the same noise as the 14-qubit workload), all trajectories in one
    launch with their uniforms resident in HBM, against the exact density
    matrix of the same circuit on the same GPU."""
    import numpy as np
    from workloads import traj_grid_circuit, uniforms
    n = 12
    ops = traj_grid_circuit()
    n_gates = sum(1 for k, _, _ in ops if k in ("su2", "cz"))
    t0 = time.perf_counter()
    prog = vqd.Trajectories(n, ops).compile()
    info = prog.info()
    nch = info["n_channels"]
    U = torch.as_tensor(uniforms(n_traj, nch), device="cuda")
    z = torch.empty((n_traj, n), dtype=torch.float64, device="cuda")
    log("trajectories: setup %.1f s, %s" % (time.perf_counter() - t0, info))
    stream = torch.cuda.current_stream()
    prog.run(U, z_out=z, norm=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        prog.run(U, z_out=z, norm=False)
    e1.record(stream)
    torch.cuda.synchronize()
    t_run = e0.elapsed_time(e1) / 1e3 / steps
    mean, sem = vqd.Trajectories.stats(z)
    mean, sem = mean.cpu().numpy(), sem.cpu().numpy()
    # the exact answer: the density-matrix path on the same circuit
    dprog = vqd.Program(n, ops).compile(vqd.plan_opts(**PLAN_OPTS))
    dm = vqd.DensityMatrix(n)
    dm.init_zero()
    dprog.run(dm)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        dm.init_zero()
        dprog.run(dm)
    e1.record(stream)
    torch.cuda.synchronize()
    t_dm = e0.elapsed_time(e1) / 1e3 / steps
    exact = dm.expec_z()
    err = float(np.abs(mean - exact).max())
    sigma = float(sem.max() * math.sqrt(n_traj))          # per-trajectory standard deviation
    need = int(math.ceil((3.0 * sigma / 1e-2) ** 2))       # 3 standard errors below 1e-2
    rate = n_traj / t_run
    tflops = 2.0 * info["fma_per_amp"] * (1 << n) * n_traj / t_run / 1e12
    out = {"metric": "noisy trajectories per second (12-qubit state vectors, one launch)",
           "workload": "2x6 grid, 2000 SU(2)/CZ gates with depol2, ZZ crosstalk and T1/T2 noise "
                       "(%d ops, %d channels); %d trajectories" % (len(ops), nch, n_traj),
           "trajectories_per_s": round(rate, 1), "ms_per_launch": round(t_run * 1e3, 3),
           "gates_per_s": round(n_gates * rate, 1), "ops_per_s": round(len(ops) * rate, 1),
           "phases": info["n_phases"], "kernel_ops": info["n_kernel_ops"],
           "planned_fp64_fma_per_amp": round(info["fma_per_amp"], 1),
           "alu": {"bound": "alu", "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(tflops / FP64_PEAK_TFLOPS, 4)},
           "max_abs_dz_vs_density_matrix": err, "max_standard_error": float(sem.max()),
           "trajectories_for_3sigma_below_1e-2": need,
           "time_to_1e-2_s": round(need / rate, 4), "density_matrix_s": round(t_dm, 5),
           "memory_per_sample_bytes": {"trajectory": 16 << n, "density_matrix": 16 << (2 * n)}}
    if oracle_sample:
        from oracle import trajectories as tj
        t0 = time.perf_counter()
        tj.run(n, ops, uniforms(1, nch)[0])
        out["oracle_trajectories_per_s"] = round(1.0 / (time.perf_counter() - t0), 3)
    del U, z, dm
    torch.cuda.empty_cache()
    return out


def device_leg(vqd):
    """Host-side noise insertion: the 2000 ideal gates of the 14-qubit grid
    circuit through a superconducting-like device specification."""
    ops, _ = workload()
    ideal = [op for op in ops if op[0] in ("su2", "cz")]
    dev = vqd.Device(N_QUBITS)
    dev.set_gate("su2", 0.05, 1e-3, 5e-4)
    dev.set_gate("cz", 0.5, 5e-3, 1e-3)
    dev.set_passive([100.0] * N_QUBITS, [50.0] * N_QUBITS)
    dev.set_crosstalk([(a, a + 1) for a in range(13) if a != 6] + [(a, a + 7) for a in range(7)], 0.01)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        noisy = dev.insert_noise(ideal)
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "2000 ideal SU(2)/CZ gates of the 14-qubit grid circuit -> %d noisy ops" % len(noisy),
            "ms_per_circuit": round(dt * 1e3, 3), "gates_per_s": round(len(ideal) / dt, 1),
            "note": "host only, including the binding's argument marshalling"}


def measure_leg(vqd, torch, dm, steps: int):
    """Measurement on the 14-qubit state the main leg leaves: projective Z
    measurement (weights, draw, collapse) and 2^20 shots from the diagonal."""
    import numpy as np
    n = dm.n
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    saved = dm.buffer.clone()
    q = n // 2
    # collapse alone: the kernel time of one measurement, from the library's
    # own launch (the weights are reduced first and come back to the host)
    t_meas = []
    for _ in range(max(1, steps)):
        dm.buffer.copy_(saved)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m, w = dm.measure_z(q, 0.25)
        torch.cuda.synchronize()
        t_meas.append(time.perf_counter() - t0)
    shots = 1 << 20
    U = torch.as_tensor(np.random.default_rng(7).random(shots), device="cuda")
    out = torch.empty(shots, dtype=torch.int32, device="cuda")
    dm.sample(U, out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(max(1, steps)):
        dm.sample(U, out)
    e1.record(stream)
    torch.cuda.synchronize()
    t_shots = e0.elapsed_time(e1) / 1e3 / max(1, steps)
    dm.buffer.copy_(saved)
    amps = 4 ** n
    # algorithmic bytes of the collapse: the quarter of the elements in the
    # support read, every element written (16 B each)
    coll_bytes = 16.0 * amps * (0.25 + 1.0)
    return {"workload": "14-qubit grid-circuit state: measure_z(q=%d) and %d shots" % (q, shots),
            "measure_z_ms": round(min(t_meas) * 1e3, 3), "outcome": m, "weight": w,
            "collapse_algorithmic_bytes": coll_bytes,
            "shots_per_s": round(shots / t_shots, 1), "sample_ms": round(t_shots * 1e3, 3)}


def surrogate_leg(vqd, torch, n_train: int, n_test: int, epochs: int):
    """The learned surrogate of the 10-qubit, 4-layer ansatz (8 device
    parameters + 16 angles -> 10 <Z_i>): training data from the batched
    emulator, training by the library's kernels, then evals/s with fallback
    against the emulator alone on a held-out set, judged by the emulator at
    |dZ| < 1e-2.  The fallback threshold is the product default, calibrated
    by the emulator on a validation set; the configured fixed threshold
    (spread >= 5e-3 falls back) is reported beside it with the accuracy of
    what it accepts.  A device-parameter sweep at fixed angles is reported
    beside the uniform-angle workload."""
    import numpy as np
    from paper_2306_07342_amd.surrogate import SurrogateModel, TemplateEmulator, measure_gain
    from workloads import SEED_BASE, c5_draw_samples, c5_params, c5_structure
    from workloads.surrogate import c5_features, init_ensemble
    st = c5_structure()
    emu = TemplateEmulator(10, st)
    # tile shape of the ansatz template from the batched autotuner (cached)
    tuned = os.path.exists(C5_TUNE_FILE)
    d0, a0 = c5_draw_samples(1024, seed=SEED_BASE + 10)
    emu.autotune(c5_params(st, d0, a0), C5_TUNE_FILE if tuned else os.path.join("/tmp", "vqd_c5_tiles.json"))

    def data(count, seed, fixed_angles=None):
        dev, ang = c5_draw_samples(count, seed=seed)
        if fixed_angles is not None:
            ang[:] = fixed_angles
        return c5_params(st, dev, ang), torch.as_tensor(c5_features(dev, ang), device="cuda")

    def run(n_tr, n_te, ep, seeds, fixed=None):
        P, x = data(n_tr, seeds[0], fixed)
        # warm-up outside the timed region: one chunk, which also sets up the
        # emulator's device buffers
        emu.run(P[:emu.chunk])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = emu.run(P).float().contiguous()
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        gpu_data, idle_data = emu.last_gpu_s, emu.last_idle_s
        log("surrogate: %d training samples in %.1f s" % (n_tr, t_data))
        model = SurrogateModel(init_ensemble(), max_batch=1024)
        t0 = time.perf_counter()
        model.fit(x, y, epochs=ep, batch=512, lr=1e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        log("surrogate: %d epochs in %.1f s, loss %s" % (ep, t_train, model.history[-1]))
        Pt, xt = data(n_te, seeds[1], fixed)
        # the emulator as judge: calibrate the spread threshold on a held-out
        # validation set so that accepted answers stay within |dZ| < 1e-2
        # (the product default); then measure on the test set with it
        Pv, xv = data(max(1024, n_te // 4), seeds[2], fixed)
        model.calibrate(xv, emu.run(Pv), tol=1e-2)
        res = measure_gain(model, emu, Pt, xt, tol=1e-2)
        res["threshold_source"] = "calibrated on %d validation samples by the emulator" % Pv.shape[0]
        fx = measure_gain(model, emu, Pt, xt, threshold=5e-3, tol=1e-2)
        res["at_configured_5e-3"] = {k: fx[k] for k in ("surrogate_evals_per_s", "surrogate_good_evals_per_s",
                                                         "gain_at_tol", "fallback_fraction",
                                                         "accepted_within_tol_fraction", "max_abs_dz_accepted",
                                                         "median_abs_dz_accepted")}
        res.update({"train_samples": n_tr, "data_gen_s": round(t_data, 2),
                    "data_gen_evals_per_s": round(n_tr / t_data, 1),
                    "data_gen_batched_kernel_only_evals_per_s": round(n_tr / gpu_data, 1),
                    "data_gen_device_idle_between_chunks_s": round(idle_data, 3),
                    "epochs": ep, "batch": 512,
                    "train_s": round(t_train, 2), "final_train_mse": [float(v) for v in model.history[-1]]})
        return res

    out = {"metric": "surrogate vs emulator evals/s at |dZ|<1e-2 (10-qubit 4-layer ansatz)",
           "config": "8 device parameters + 16 angles drawn uniformly, 4 x MLP 24-256-256-256-10 GELU, "
                     "bf16 operands / FP32 accumulate; fallback above an emulator-calibrated spread "
                     "threshold (the configured 5e-3 reported beside it)"}
    out["template_tiles"] = {"tile_bits": emu.opts.tile_bits, "min_contig_bits": emu.opts.min_contig_bits,
                             "source": "autotuned (%s)" % ("cached" if tuned else "fresh")}
    out["uniform_angles"] = run(n_train, n_test, epochs, (SEED_BASE + 4, SEED_BASE + 6, SEED_BASE + 11))
    fixed = c5_draw_samples(1, seed=SEED_BASE + 7)[1][0]
    out["device_sweep_fixed_angles"] = run(max(4096, n_train // 8), max(1024, n_test // 4), 4 * epochs,
                                           (SEED_BASE + 8, SEED_BASE + 9, SEED_BASE + 12), fixed)
    emu.release()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-every", type=int, default=180)   # ~52 ops, 10-15 s of oracle work
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-emulation leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-16q", action="store_true", help="skip the 16-qubit context leg")
    ap.add_argument("--no-traj", action="store_true", help="skip the trajectory leg")
    ap.add_argument("--no-measure", action="store_true", help="skip the measurement leg")
    ap.add_argument("--trajectories", type=int, default=1 << 16, help="trajectories per launch")
    ap.add_argument("--surrogate-train", type=int, default=1 << 18, help="training samples (2^18)")
    ap.add_argument("--surrogate-test", type=int, default=1 << 14, help="held-out samples (2^14)")
    ap.add_argument("--surrogate-epochs", type=int, default=30)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device-to-device copy of the state buffer "
                         "(known size) for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(how it would shard is documented with the design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_07342_amd import vqd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ops, n_gates = workload()
    n = N_QUBITS
    log("planning %d ops (%d gates) on %d qubits" % (len(ops), n_gates, n))
    t = time.perf_counter()
    prog = vqd.Program(n, ops).compile(vqd.plan_opts(**PLAN_OPTS))
    info = prog.info()
    log("plan: %s (%.2f s)" % (info, time.perf_counter() - t))
    dm = vqd.DensityMatrix(n)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        dm.init_zero()
        if ev:
            ev[0].record(stream)
        prog.run(dm)
        if ev:
            ev[1].record(stream)
        z = dm.expec_z()
        pur = dm.purity()
        return z, pur

    for w in range(args.warmup):
        step()
        log("warmup %d done" % w)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        z, pur = step(evs[k])
        log("step %d done" % k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    tr = dm.trace()
    if args.calibrate_copy:
        y = torch.empty_like(dm.buffer)
        y.copy_(dm.buffer)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (dm.buffer.numel() * 8, y.numel() * 8))
        del y

    amps = 4 ** n
    bytes_per_pass = pass_bytes(info, amps) / info["n_passes"]     # average over the launches
    avg_launch_s = pass_ms / 1e3 / info["n_passes"]
    achieved_gbs = bytes_per_pass / avg_launch_s / 1e9
    fp64_tflops = executed_flops(info, amps) / (pass_ms / 1e3) / 1e12
    traffic = measured_traffic()
    hbm = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    alu = {"bound": "alu", "achieved": round(fp64_tflops, 2), "peak": FP64_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(fp64_tflops / FP64_PEAK_TFLOPS, 4), "traffic": traffic}
    roof = hbm if hbm["frac"] >= alu["frac"] else alu

    ms_per_step = wall / args.steps * 1e3
    out = {
        "metric": METRIC,
        "value": round(len(ops) * args.steps / wall, 1),
        "unit": "DM ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "14-qubit density matrix (complex128, 4^14 amps), 2x7 grid, "
                               "2000-gate layered SU(2)+CZ circuit with depol2, ZZ crosstalk and T1/T2 noise",
                   "n_qubits": n, "dm_ops_per_step": len(ops), "gates_per_step": n_gates,
                   "seed": 2306073421, "parallelism": "single GPU"},
        "gates_per_s": round(n_gates * args.steps / wall, 1),
        "passes_per_step": info["n_passes"],
        "phases_per_step": info["n_phases"],
        "hermitian_mode": bool(info["hermitian"]),
        "relabelled_layouts": bool(info["relabelled"]),
        "computed_tile_fraction": round(info["tile_fraction"], 6),
        "planned_fp64_fma_per_amp": round(info["fma_per_amp"], 1),
        "executed_fp64_fma_per_amp": round(info["fma_per_amp"] * info["tile_fraction"], 1),
        "bytes_per_launch": round(bytes_per_pass, 1),
        # executed FP64 flops per algorithmic HBM byte; the FP64 ridge is
        # 78.6 TFLOP/s / 8 TB/s = 9.8 flop/B
        "flop_per_byte": round(executed_flops(info, amps) / (bytes_per_pass * info["n_passes"]), 2),
        "pass_kernel_ms_per_step": round(pass_ms, 3),
        "pass_kernel_avg_launch_us": round(avg_launch_s * 1e6, 2),
        "roofline": roof,
        "roofline_other": alu if roof is hbm else hbm,
        # context, not a roofline: the bytes an op-by-op path (one HBM pass
        # per density-matrix op) would move, per second of the fused path
        "unfused_equivalent_gbs": round(32.0 * amps * len(ops) * args.steps / wall / 1e9, 1),
        "check": {"trace_re": tr.real, "purity": pur, "z0": float(z[0])},
    }
    out["device_layer"] = device_leg(vqd)
    if not args.no_measure:
        log("measurement leg ...")
        out["measurement"] = measure_leg(vqd, torch, dm, args.steps)
    if not args.no_batched:
        log("batched leg ...")
        out["batched"] = batched_leg(vqd, torch, args.steps)
    if not args.no_traj:
        log("trajectory leg ...")
        out["trajectories"] = traj_leg(vqd, torch, args.trajectories, args.steps, not args.no_cpu_baseline)
    if not args.no_16q and torch.cuda.get_device_properties(0).total_memory > 100 * 2 ** 30:
        log("16-qubit leg ...")
        del dm
        torch.cuda.empty_cache()
        out["c3_16q"] = c3_leg(vqd, torch, 1)
    if not args.no_surrogate:
        log("surrogate leg ...")
        out["surrogate"] = surrogate_leg(vqd, torch, args.surrogate_train, args.surrogate_test,
                                         args.surrogate_epochs)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(ops, n, args.cpu_sample_every)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
