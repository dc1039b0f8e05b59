import decimal
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Oracle points are 100-digit Decimals; arithmetic on them in the tests (differences,
# negations) must not round to the 28-digit default context.
decimal.getcontext().prec = 120


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def lib():
    """The loaded HIP library binding (GPU tests only)."""
    from paper_2510_09892_amd import sphint
    return sphint.load()
