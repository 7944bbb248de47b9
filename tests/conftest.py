import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU case")


@pytest.fixture(scope="session")
def configs():
    """Cache of generated synthetic configurations, keyed by number."""
    import meshgen
    cache = {}

    def get(k):
        if k not in cache:
            cache[k] = meshgen.make_config(k)
        return cache[k]
    return get
