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


def pytest_sessionstart(session):
    """Build the libraries once if this checkout has none (they are not committed)."""
    pkg = os.path.join(ROOT, "paper_2510_09892_amd")
    libs = [os.path.join(pkg, n) for n in ("libsphint.so", "libsphint_hostcheck.so")]
    if not all(os.path.exists(p) for p in libs):
        from paper_2510_09892_amd import build
        build.build()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def lib():
    """The loaded HIP library binding (GPU tests only)."""
    from paper_2510_09892_amd import sphint
    return sphint.load()
