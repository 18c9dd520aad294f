"""The binding on a fresh process: the library may be the first to touch the
GPU (PyTorch's runtime is brought up before the library's kernels are
registered), and device tensors still work afterwards."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
from paper_2306_07342_amd import vqd
from workloads import c5_draw_samples, c5_params, c5_structure
st = c5_structure(n=4, layers=1)
dev, ang = c5_draw_samples(3, seed=1, n_angles=4)
b = vqd.Batch()                           # first GPU use in this process
t = b.add_template(4, [(k, q) for k, q, _ in st])
b.add_instances(t, c5_params(st, dev, ang))
b.compile()
b.run()
import torch
x = torch.ones(8, device="cuda") * 2
assert float(x.sum()) == 16.0
print("ok", b.expec_z(0).shape)
"""


def test_library_first_then_torch_in_fresh_process():
    r = subprocess.run([sys.executable, "-c", CHILD % ROOT], capture_output=True, text=True, timeout=180)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0 and "ok" in r.stdout
