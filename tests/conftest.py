import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle():
    from oracle import helm_oracle

    helm_oracle.lib()
    return helm_oracle


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Print the case name before every GPU test so a fault can be attributed."""
    if request.node.get_closest_marker("gpu") is not None:
        print(f"\n[gpu-case] {request.node.nodeid}", file=sys.stderr, flush=True)
    yield
