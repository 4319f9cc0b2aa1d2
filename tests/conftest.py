import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library on a visible GPU; the product path has no CPU fallback."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    torch.cuda.init()
    from paper_1401_0782_amd import _abi

    return _abi.load()


@pytest.fixture(autouse=True)
def _gpu_runtime_first(request):
    """Every GPU test brings up torch's GPU runtime before the library's first
    call (a test selected on its own, without gpu_lib, would otherwise let the
    library initialise HIP first, after which torch reports no GPU)."""
    if request.node.get_closest_marker("gpu"):
        request.getfixturevalue("gpu_lib")
