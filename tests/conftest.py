import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


import pytest  # noqa: E402


def _gpu_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_ok():
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    # name the case before any GPU work, so a crash log says which one ran;
    # start from cleared sticky statuses (a case that provoked a
    # non-physical state on purpose leaves its flag for the next check)
    if "gpu" in request.keywords:
        print(f"\n[gpu case] {request.node.nodeid}", flush=True)
        from paper_2502_02704_amd import bgk
        if bgk._lib is not None:
            bgk.status()
    yield
