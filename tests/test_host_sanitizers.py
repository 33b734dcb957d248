"""Host code under the sanitizers, on the CPU (no device call is made):

  * the CPU oracle (oracle/dbg_oracle.c) driven by tests/host/oracle_sanitize.c
    under AddressSanitizer and UndefinedBehaviorSanitizer;
  * the runtime's host logic (tests/host/host_logic.cpp, which includes the
    runtime header) under the same two, built with hipcc for its host part;
  * the threaded CPU build of the paper's lock-free design
    (oracle/lfdbg_cpu.cpp) driven by tests/host/lfdbg_tsan.cpp under
    ThreadSanitizer, 8 threads racing on one and on 64 list heads.

Each program must exit 0, print "ok" and leave no sanitizer report."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
REPORT = ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer")


def _run(cmd_build, exe, env=None):
    b = subprocess.run(cmd_build, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert r.stdout.strip().endswith("ok"), out[-3000:]
    for marker in REPORT:
        assert marker not in out, out[-3000:]


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(HOST, "oracle_sanitize.c"),
          os.path.join(ROOT, "oracle", "dbg_oracle.c")], exe)


def test_host_logic_under_asan_ubsan(tmp_path):
    hipcc = next((c for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc"))
                  if c and os.path.exists(c)), None)
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "host_logic_san")
    # sanitizers on the host part only (each -fsanitize= right after -Xarch_host)
    _run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all",
          "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2401_02756_amd", "csrc"),
          "-o", exe, os.path.join(HOST, "host_logic.cpp")], exe)


def test_lfdbg_threads_under_tsan(tmp_path):
    exe = str(tmp_path / "lfdbg_tsan")
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-pthread", "-o", exe,
          os.path.join(HOST, "lfdbg_tsan.cpp"), os.path.join(ROOT, "oracle", "lfdbg_cpu.cpp")], exe, env)
