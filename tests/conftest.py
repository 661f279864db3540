import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _ensure_built():
    """Build the oracle and the host generator only when nothing is built."""
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()
    from paper_0807_0264_amd import synth
    if not os.path.exists(synth.CPU_LIB):
        synth.build()


_ensure_built()


@pytest.fixture(scope="session")
def O():
    from oracle import oracle
    return oracle


@pytest.fixture(scope="session")
def S():
    from paper_0807_0264_amd import synth
    return synth
