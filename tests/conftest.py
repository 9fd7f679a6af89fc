import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_table():
    """The oracle's 2^32 odd-only sieve table (256 MiB), built once."""
    import oracle
    return oracle.table()


def golden(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    return [line.rstrip("\n") for line in open(path) if line.strip() and not line.startswith("#")]
