"""Host-side pieces of the benchmark line (no GPU): the committed counter
profiles' code digest, which decides whether the line reports HBM traffic."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_digest_ignores_comments_but_not_code(tmp_path):
    a = tmp_path / "a.hip"
    a.write_text("// header\nint f(int x) {  /* twice */\n    return 2 * x;  // doubled\n}\n")
    b = tmp_path / "b.hip"
    b.write_text("\n\nint f(int x) {\n  return 2 * x;\n}\n/* a longer\n   comment */\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x) {\n    return 3 * x;\n}\n")
    assert bench.code_digest([str(a)]) == bench.code_digest([str(b)])
    assert bench.code_digest([str(a)]) != bench.code_digest([str(c)])



def test_committed_traffic_needs_the_recorded_workload():
    """A profile's traffic is reported only for the workload parameters it
    records (here a load factor it was not taken at)."""
    assert bench.committed_traffic("hbm_traffic_large_c3.md", {"workload": "large_c3", "load_factor": 0.4,
                                                               "mode": "binned", "entry_bytes": 24}, "k_reduce") is None
    assert bench.committed_traffic("no_such_profile.md", {}, "k_reduce") is None
