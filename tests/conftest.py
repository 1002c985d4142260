import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def lut9():
    import oracle
    return oracle.build_lut(9)


@pytest.fixture(scope="session")
def scene_c0():
    from paper_2609_36267_amd import synth
    return synth.config("c0", keep_truth=True)
