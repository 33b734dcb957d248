"""Host-side logic of the runtime on the CPU: the binned table geometry, the
size classes that key captured passes, and dbg_build's host count of
windows and k-mers (tests/host/host_logic.cpp, compiled here with hipcc and
run without a device).  No GPU call is made."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_logic(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "host_logic")
    cmd = [hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2401_02756_amd", "csrc"),
           "-o", exe, os.path.join(ROOT, "tests", "host", "host_logic.cpp")]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), run.stdout[-2000:]
