import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def golden():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as f:
        return json.load(f)


@pytest.fixture(scope="session", autouse=True)
def _torch_runtime_first(request):
    """When GPU tests are selected, start torch's HIP runtime before the
    library's, the order bench.py uses: torch's first use after the library
    had run large searches has failed to find the device."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        import torch
        if torch.cuda.is_available():
            torch.zeros(1, device="cuda:0")
    yield
