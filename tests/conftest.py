import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size workloads (minutes)")


def _ensure_host_libs():
    # Build the host-side libraries only when nothing is built yet.
    import oracle
    import synth
    if not os.path.exists(synth.lib_path()):
        synth.build_lib()
    if not os.path.exists(oracle.lib_path()):
        oracle.build_lib()


_ensure_host_libs()


@pytest.fixture(scope="session")
def root():
    return ROOT
