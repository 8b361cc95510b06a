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
    """The HIP library through its Python binding; GPU tests only."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_10899_amd import _lib
    return _lib.load()


@pytest.fixture(autouse=True, scope="module")
def _release_library_caches(request):
    """After each GPU test module, drop the library's cached plans and
    workspaces, so that the modules do not accumulate device memory."""
    yield
    marks = getattr(request.module, "pytestmark", [])
    marks = marks if isinstance(marks, list) else [marks]
    if not any(getattr(m, "name", "") == "gpu" for m in marks):
        return
    lib = sys.modules.get("paper_1710_10899_amd._lib")
    if lib is not None and getattr(lib, "_lib", None) is not None:
        lib.submat_release()
