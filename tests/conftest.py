import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~10 s")


@pytest.fixture(autouse=True)
def _scratch_returned():
    """After every test: each library call returns what it took from the
    binding's scratch workspaces (a leak would shrink them for later calls)."""
    yield
    mcd = sys.modules.get("paper_2509_22975_amd")
    if mcd is None or not getattr(mcd, "_SCRATCH", None):
        return
    for key, ws in list(mcd._SCRATCH.items()):
        if ws.handle:
            used = ws.stats()["in_use"]
            assert used == 0, f"scratch workspace {key} still holds {used} bytes after the test"
