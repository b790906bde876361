import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    # The oracle and the input generator are plain C built with gcc; build them if absent.
    import graphgen
    import oracle
    if not os.path.exists(graphgen._LIB):
        graphgen.build(force=False)
    if not os.path.exists(oracle._LIB):
        oracle.build(force=False)
    yield
