import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: large inputs (minutes of CPU)")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    # Build the generator and oracle libraries only if nothing is built yet.
    import gen
    import oracle
    gen.build(force=False)
    oracle.build(force=False)
    yield
