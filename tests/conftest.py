import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libhsdm.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    return O


_ORACLE_RUNS = {}


@pytest.fixture(scope="session")
def oracle_run():
    """run(key, fn): fn() once per session (an oracle solve at a size that
    takes tens of seconds on the host), cached by key.  Progress goes to the
    real stderr so that a long oracle run is not silent under capture."""
    import time

    def run(key, fn):
        if key not in _ORACLE_RUNS:
            t0 = time.time()
            print(f"[oracle] {key}: start", file=sys.__stderr__, flush=True)
            _ORACLE_RUNS[key] = fn()
            print(f"[oracle] {key}: {time.time() - t0:.1f} s", file=sys.__stderr__, flush=True)
        return _ORACLE_RUNS[key]

    return run
