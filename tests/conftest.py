import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: larger CPU-only case")


@pytest.fixture(scope="session")
def small_pair():
    from paper_2206_03410_amd import synth
    return synth.torus_pair(1000, n_src=400, n_tgt=400, n_nodes=24, k=4, e=6)


@pytest.fixture(scope="session")
def small_prob(small_pair):
    from oracle import amm_oracle as O
    return O.from_pair(small_pair)
