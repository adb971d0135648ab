import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def mech_small():
    import oracle
    from synth import mechanism_file
    return oracle.load_mechanism(mechanism_file("h2like_10_27"))


@pytest.fixture(scope="session")
def mech_tiny():
    import oracle
    from synth import mechanism_file
    return oracle.load_mechanism(mechanism_file("tiny_8_14"))


@pytest.fixture(scope="session")
def mech_methane():
    import oracle
    from synth import mechanism_file
    return oracle.load_mechanism(mechanism_file("ch4like_53_325"))
