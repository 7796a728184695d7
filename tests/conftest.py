import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def cfg1():
    from paper_1912_05529_amd import synth
    return synth.config1()


@pytest.fixture(scope="session")
def cfg1_table(cfg1):
    import oracle
    return oracle.design_table(cfg1.desc)


@pytest.fixture(scope="session")
def cfg2_model():
    from paper_1912_05529_amd import synth
    return synth.config2(with_data=False)


@pytest.fixture(scope="session")
def cfg2_table(cfg2_model):
    import oracle
    return oracle.design_table(cfg2_model.desc)
