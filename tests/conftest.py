import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "libmpm_oracle.so")):
        oracle.build(force=True)
    return oracle


def observations(orc, case, use_b1=True):
    """x = s(truth) + sigma * eps as float32 values widened to float64, i.e. the
    exact numbers the GPU library is given."""
    s = orc.simulate(case["proto"], case["truth"], case["b1"] if use_b1 else None)
    x = (s + case["sigma"] * case["eps"].astype(np.float64)).astype(np.float32)
    return x


def sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))
