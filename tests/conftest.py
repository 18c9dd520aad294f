import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, loaded through its Python binding (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2306_07342_amd import vqd
    vqd.load()
    return vqd


@pytest.fixture(scope="session")
def vqd_host():
    """The library loaded for host-only use (planning, builders); built if missing."""
    from paper_2306_07342_amd import build as vbuild, vqd
    import os
    if not os.path.exists(vqd.LIB_PATH):
        vbuild.build()
    vqd.load()
    return vqd
