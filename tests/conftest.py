import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-only case")


def pytest_collection_modifyitems(config, items):
    # keep GPU tests in a fixed, cheap-first order inside each file
    pass


@pytest.fixture(scope="session")
def cfg1_problem():
    import synth
    from oracle import bse
    return bse.make_problem(synth.config("cfg1"))


@pytest.fixture(scope="session")
def cfg1_h(cfg1_problem):
    from oracle import bse
    return bse.hamiltonian(cfg1_problem)
