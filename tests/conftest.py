import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_capture = None


def pytest_configure(config):
    global _capture
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    _capture = config.pluginmanager.getplugin("capturemanager")


def say(*a):
    """Progress line of a GPU test, written past pytest's output capture: it
    names the case before each GPU step and shows that a long test is alive."""
    msg = " ".join(str(x) for x in ("[case]",) + a)
    if _capture is not None:
        with _capture.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


@pytest.fixture(scope="session")
def oracle_native():
    from oracle import native
    native.build(force=False)
    return native
