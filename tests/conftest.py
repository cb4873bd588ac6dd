import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")
    config.addinivalue_line("markers", "slow: longer CPU checks")


@pytest.fixture(scope="session")
def mask_m1():
    """32^3 bicontinuous mask, lambda = 8 voxels, phi = 0.70, mask seed 0."""
    from paper_2604_13929_amd import inputs
    return inputs.spinodal_mask(32, 32, 32, 8.0, 0.70, seed=0)


GOLDEN = os.path.join(TESTS, "golden")


def golden(name: str):
    """Rows of a cited text fixture under tests/golden/ ('#' lines are the citation)."""
    import numpy as np
    return np.atleast_2d(np.loadtxt(os.path.join(GOLDEN, name), comments="#"))
