import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: longer CPU test (oracle at larger chi)")


@pytest.fixture(scope="session", autouse=True)
def _torch_runtime_first(request):
    """torch carries its own HIP runtime: when GPU tests run, let it find the device before the
    library's runtime opens it in this process (the other order leaves torch without a device)."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
    yield
