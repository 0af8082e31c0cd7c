import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def tiny_cfg():
    from synth import cfg_tiny
    return cfg_tiny()


@pytest.fixture(scope="session")
def tiny_iq(tiny_cfg):
    """Oracle-simulated channel data of ensemble 0 of the tiny configuration."""
    from synth import make_medium
    from oracle import sim
    med = make_medium(tiny_cfg, 0)
    return sim.simulate(tiny_cfg, med)
