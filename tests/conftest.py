import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# Parity tests run the library with its stage-by-stage index validation on:
# an inconsistent intermediate array becomes an error, not a bad access.
os.environ.setdefault("JP_CHECKS", "1")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(params=["checked", "shipped"])
def checks_mode(request):
    """Runs a test twice: with the library's stage-by-stage validation of
    intermediate index arrays on ("checked") and off, as shipped and timed
    ("shipped")."""
    import ctypes
    import paper_2002_12459_amd as jp
    lib = jp._load()
    lib.jp_test_set_checks.argtypes = [ctypes.c_int32]
    lib.jp_test_set_checks.restype = ctypes.c_int32
    prev = lib.jp_test_set_checks(1 if request.param == "checked" else 0)
    try:
        yield request.param
    finally:
        lib.jp_test_set_checks(prev)


def load_golden(name):
    """Parse a fixture under tests/golden: '#' comments, whitespace fields."""
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows
