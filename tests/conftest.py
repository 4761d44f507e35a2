import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


def ensure_hip_lib():
    """Build libhpic.so in-tree if it is not there (hipcc cross-compiles on CPU)."""
    from paper_1502_01376_amd import hpic
    if not os.path.exists(hpic.LIBPATH):
        from paper_1502_01376_amd.csrc import build
        build.build()
    return hpic


@pytest.fixture(scope="session")
def hpic():
    """The library binding on a machine with a GPU (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01376_amd import hpic as mod
    if not os.path.exists(mod.LIBPATH):
        raise RuntimeError("libhpic.so is not built: the GPU tests need the HIP library")
    return mod
