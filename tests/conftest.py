import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.build(force=False)
    return O


@pytest.fixture(scope="session")
def c1():
    from paper_1110_4372_amd import synth
    return synth.make_catalog("c1", seed=0)


@pytest.fixture(scope="session")
def c1_oracle(orc, c1):
    p = orc.params_of(c1)
    return orc.run_all(p, orc.Particles.of(c1))


@pytest.fixture(scope="session")
def c2():
    from paper_1110_4372_amd import synth
    return synth.make_catalog("c2", seed=0)


@pytest.fixture(scope="session")
def c2_fof_oracle(orc, c2):
    """The oracle's FOF labels of the 128^3 catalogue."""
    return orc.fof3d(orc.params_of(c2), orc.Particles.of(c2))
