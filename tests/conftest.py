import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    # the autotuner's cache file: one per test session, never the user's
    if "DBG_TUNE_CACHE" not in os.environ:
        import tempfile
        os.environ["DBG_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="dbg_tune_"), "autotune.tsv")
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: large inputs; minutes of CPU")


def read_golden(name):
    """Non-comment lines of a golden fixture, split into fields."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def worked_example():
    rows = read_golden("worked_example_acgacgacgc_k4.txt")
    read = [r[1] for r in rows if r[0] == "read"][0]
    k = int([r[1] for r in rows if r[0] == "k"][0])
    verts = {r[1]: (int(r[2]), [int(x) for x in r[3:7]]) for r in rows if r[0] == "vertex"}
    return read, k, verts
