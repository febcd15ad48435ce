import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    # GPU tests need a device; on a machine without one they are skipped rather
    # than failing, so `-m "not gpu"` and a plain run both work on CPU hosts.
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def nproc():
    return min(16, os.cpu_count() or 1)


@pytest.fixture(scope="session")
def oracle_pool(nproc):
    """2048 oracle points P_i = k_i G (k_i from the shared seeded generator)."""
    from oracle import points
    from paper_2502_11660_amd import inputs
    kw = inputs.nonzero_scalars_mod_r(inputs.config_seed(1), 2048, stream=7)
    ks = [inputs.words_to_int(r) for r in kw]
    # serial on purpose: no worker processes forked from a process that may
    # already hold a GPU context
    pts = points.gen_points(ks)
    return ks, pts
