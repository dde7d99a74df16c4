import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


_capman = None


def pytest_configure(config):
    global _capman
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    _capman = config.pluginmanager.getplugin("capturemanager")


def progress(msg: str) -> None:
    """Print a progress line past pytest's output capture, so that long GPU
    tests show that they are working while they run."""
    if _capman is not None:
        with _capman.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build()
    yield
