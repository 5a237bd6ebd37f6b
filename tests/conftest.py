import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (large oracle runs)")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """The generator and oracle are plain C; build them if this checkout has no .so yet."""
    import oracle
    import synth

    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    yield
