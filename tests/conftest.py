import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _native_builds():
    """Compile the checker and the input generator (plain gcc, seconds) if they are absent."""
    import oracle
    import workloads
    oracle.build_native(force=False)
    workloads.build_native(force=False)
