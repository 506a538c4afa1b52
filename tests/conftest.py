import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(1234)


def pytest_collection_modifyitems(config, items):
    # import torch once at collection so the first GPU test does not pay for it
    if any(item.get_closest_marker("gpu") for item in items):
        try:
            import torch  # noqa: F401
        except Exception:
            pass
