import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size GPU parity case")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; on a host without one they are skipped,
    # never silently routed elsewhere.
    try:
        import torch

        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def sess():
    """One library context per test session (GPU tests only)."""
    from paper_1702_03484_amd.engine import MapSQ

    s = MapSQ(arena_bytes=48 << 30)
    yield s
    s.close()


def announce(msg: str):
    """Name the GPU case before it runs (flushed, so a crash still shows it)."""
    print(f"\n[gpu-case] {msg}", flush=True)
