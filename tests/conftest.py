import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


_instances = {}


def cached_instance(name, n=None, absent=False):
    """Session-wide cache of oracle-built PIR instances (keys, database, encrypted query)."""
    import datagen
    from oracle.client import build_instance
    key = (name, n, absent)
    if key not in _instances:
        cfg = datagen.CONFIGS[name] if isinstance(name, str) else name
        _instances[key] = build_instance(cfg, n=n, absent=absent)
    return _instances[key]


@pytest.fixture(scope="session")
def instances():
    return cached_instance
