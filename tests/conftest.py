import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    so = ROOT / "oracle" / "liboracle.so"
    src = ROOT / "oracle" / "rco.c"
    if not so.exists() or so.stat().st_mtime < src.stat().st_mtime:
        from oracle import build as ob
        ob.build()
    yield
