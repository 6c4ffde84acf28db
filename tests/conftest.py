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
def oracle_run(request):
    """run(key, fn): fn() once per session (an oracle solve at a size that
    takes tens of seconds on the host), cached by key.  Its progress lines
    are printed with output capture suspended, so that a long oracle run is
    not silent."""
    import time

    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        if capman is not None:
            capman.suspend_global_capture(in_=False)
        try:
            print(msg, file=sys.stderr, flush=True)
        finally:
            if capman is not None:
                capman.resume_global_capture()

    def run(key, fn):
        if key not in _ORACLE_RUNS:
            t0 = time.time()
            say(f"\n[oracle] {key}: start")
            _ORACLE_RUNS[key] = fn()
            say(f"[oracle] {key}: {time.time() - t0:.1f} s on {os.cpu_count()} host cpus")
        return _ORACLE_RUNS[key]

    return run
