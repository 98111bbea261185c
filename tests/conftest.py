import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


class _Model:
    """Minimal model description accepted by the oracle (duck-typed)."""

    def __init__(self, channel, spin, width_mode=0, lineshape=None, flatte_ratio=None):
        import synth
        self.channel = list(channel)
        self.spin = list(spin)
        self.width_mode = width_mode
        self.parent_mass = synth.PARENT_MASS
        self.masses = synth.DAUGHTER_MASSES
        self.r = synth.R_BARRIER
        self.n_res = len(self.channel)
        self.lineshape = None if lineshape is None else list(lineshape)
        self.flatte_masses = synth.FLATTE_MASSES
        self.flatte_ratio = synth.FLATTE_RATIO if flatte_ratio is None else flatte_ratio


@pytest.fixture
def make_model():
    return _Model
