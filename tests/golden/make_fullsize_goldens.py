"""Write the full-size oracle goldens of the 14-qubit grid circuit and of the
all-to-all circuit's generator at 15 qubits.  Test infrastructure.

    OMP_NUM_THREADS=8 python tests/golden/make_fullsize_goldens.py grid14 [--checkpoint DIR]
    OMP_NUM_THREADS=8 python tests/golden/make_fullsize_goldens.py a2a15  [--checkpoint DIR]

Each run applies the whole op stream on the CPU oracle (``oracle/``), one op
at a time, then stores its read-outs in ``tests/golden/<name>.json``: trace,
purity, <Z_i>, <Z_i Z_j> for every pair, every diagonal probability, and a
seeded sample of amplitudes (row r, column c, rho_{rc}).  Nothing here calls
the GPU library; the op streams come from ``workloads`` (seeded draws only).

The 14-qubit state is 4.3 GB and the 15-qubit one 17.2 GB of host memory; the
runs take hours on 8 cores.  With ``--checkpoint DIR`` the state is saved every
``--every`` ops and a restarted run resumes from the last save.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import channels  # noqa: E402
from oracle.core import OracleDM  # noqa: E402
from oracle.emulator import readouts  # noqa: E402
from workloads import c2_grid_circuit, c3_all_to_all_circuit  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name -> (qubits, op-stream factory, description)
CASES = {
    "grid14": (14, lambda: c2_grid_circuit(rows=2, cols=7, n_gates=2000),
               "2x7 grid circuit, 2000 gates (SU(2) layers, CZ + depol2, ZZ crosstalk, T1/T2)"),
    "a2a15": (15, lambda: c3_all_to_all_circuit(n=15, n_gates=500),
              "all-to-all circuit generator at 15 qubits, 500 gates (XX + depol2, Rz/Ry, deph1)"),
}
N_AMP_SAMPLES = 8192
SAMPLE_SEED = 7342


def sample_indices(n: int, count: int = N_AMP_SAMPLES, seed: int = SAMPLE_SEED):
    """Seeded (row, column) pairs: the first count/16 lie on the diagonal
    (r = c, the populations), the rest are uniform over the matrix."""
    rng = np.random.default_rng(seed + n)
    D = 1 << n
    r = rng.integers(0, D, count)
    c = rng.integers(0, D, count)
    m = count // 16
    c[:m] = r[:m]
    return r.astype(np.int64), c.astype(np.int64)


def _apply(dm: OracleDM, op) -> None:
    what, payload = channels.build(op)
    if what == "matrix":
        dm.apply_matrix(op[1], payload)
    else:
        dm.apply_kraus(op[1], payload)


def run(name: str, checkpoint: str | None, every: int) -> str:
    n, make, desc = CASES[name]
    ops = make()
    dm = OracleDM(n)
    start = 0
    ck_state = ck_meta = None
    if checkpoint:
        os.makedirs(checkpoint, exist_ok=True)
        ck_state = os.path.join(checkpoint, name + ".state.npy")
        ck_meta = os.path.join(checkpoint, name + ".json")
        if os.path.exists(ck_meta) and os.path.exists(ck_state):
            with open(ck_meta) as f:
                start = json.load(f)["next_op"]
            dm.R[...] = np.load(ck_state, mmap_mode="r")
            print("resumed %s at op %d of %d" % (name, start, len(ops)), flush=True)
    t0 = time.time()
    for i in range(start, len(ops)):
        _apply(dm, ops[i])
        done = i + 1
        if done % 50 == 0 or done == len(ops):
            el = time.time() - t0
            rate = (done - start) / el
            print("%s: %d/%d ops, %.0f s, %.2f ops/s, eta %.0f s"
                  % (name, done, len(ops), el, rate, (len(ops) - done) / rate), flush=True)
        if ck_state and done % every == 0 and done < len(ops):
            np.save(ck_state + ".tmp.npy", dm.R)
            os.replace(ck_state + ".tmp.npy", ck_state)
            with open(ck_meta, "w") as f:
                json.dump({"next_op": done}, f)
    ro = readouts(dm)
    r, c = sample_indices(n)
    amps = dm.R[r, c]
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    out = {
        "what": desc,
        "made_by": "tests/golden/make_fullsize_goldens.py %s (CPU oracle, every op in order, no fusion)" % name,
        "n": n,
        "n_ops": len(ops),
        "trace": [float(ro["trace"].real), float(ro["trace"].imag)],
        "purity": float(ro["purity"]),
        "expec_z": [float(x) for x in ro["expec_z"]],
        "pairs": pairs,
        "expec_zz": [float(x) for x in ro["expec_zz"]],
        "probs": [float(x) for x in ro["probs"]],
        "amp_seed": SAMPLE_SEED + n,
        "amp_rows": [int(x) for x in r],
        "amp_cols": [int(x) for x in c],
        "amp_re": [float(x) for x in amps.real],
        "amp_im": [float(x) for x in amps.imag],
    }
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, flush=True)
    return path


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--checkpoint", default=None, help="directory for resumable state saves")
    ap.add_argument("--every", type=int, default=1000, help="ops between state saves")
    a = ap.parse_args()
    run(a.case, a.checkpoint, a.every)
    return 0


if __name__ == "__main__":
    sys.exit(main())
