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
    from tests import gpu_util
    gpu_util.ERRORS.clear()
    yield
    if gpu_util.ERRORS:
        _MARGINS[request.node.nodeid] = (max(gpu_util.ERRORS), len(gpu_util.ERRORS))


_MARGINS = {}  # test id -> (largest normwise error measured, comparisons)


def pytest_terminal_summary(terminalreporter):
    """The parity margins: per test, the largest normwise error that its
    comparisons measured (against the oracle, or between two GPU paths),
    the 1e-12 bar being the usual one."""
    if not _MARGINS:
        return
    from tests.gpu_util import TOL
    tr = terminalreporter
    tr.section("parity margins")
    rows = sorted(_MARGINS.items(), key=lambda kv: -kv[1][0])
    n_cmp = sum(c for _, (_, c) in rows)
    tr.write_line(f"{len(rows)} tests, {n_cmp} normwise comparisons; largest errors "
                  f"(fraction of the {TOL:g} bar):")
    for nodeid, (e, c) in rows[:20]:
        tr.write_line(f"  {e:.3e}  ({e / TOL:6.3f})  {c:3d} cmp  {nodeid}")
    below = sum(1 for _, (e, _) in rows if e <= 0.1 * TOL)
    tr.write_line(f"{below} of {len(rows)} tests stay within a tenth of the bar")
