import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU reference case")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def wl5_full():
    """Workload 5 at its full pixel count (nside 512, 3 145 728 pixels, 350 polarised
    antennas), one LST and the two ends of its band: shared by the interpolated and
    the learned-beam tests (generating the sky takes several seconds)."""
    from paper_2312_09763_amd import synth
    return synth.workload(5, n_time=1, n_freq=2)
