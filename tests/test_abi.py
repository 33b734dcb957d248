"""The C-ABI library loads, exports what the header declares, and rejects bad
arguments on the host before touching a device.  Runs without a GPU."""

import ctypes
import os
import re
import subprocess

import pytest

import paper_2401_02756_amd as dbg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dbg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dbg_[a-z_]+)\s*\(", text)))


def declared_codes():
    text = open(os.path.join(ROOT, "include", "dbg.h")).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"#define DBG_(E_[A-Z]+|OK) \(?(-?\d+)\)?", text)}


def test_library_exports_every_declared_symbol():
    L = dbg.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert sorted(dbg.EXPORTS) == names


def test_binding_codes_match_header():
    codes = declared_codes()
    assert codes["OK"] == dbg.OK
    assert codes["E_INVAL"] == dbg.E_INVAL and codes["E_K"] == dbg.E_K
    assert codes["E_BASE"] == dbg.E_BASE and codes["E_NOMEM"] == dbg.E_NOMEM
    assert codes["E_FULL"] == dbg.E_FULL and codes["E_SPACE"] == dbg.E_SPACE
    assert codes["E_DEVICE"] == dbg.E_DEVICE and codes["E_RANGE"] == dbg.E_RANGE
    assert codes["E_STATE"] == dbg.E_STATE and codes["E_SCRATCH"] == dbg.E_SCRATCH
    text = open(os.path.join(ROOT, "include", "dbg.h")).read()
    assert int(re.search(r"#define DBG_PENDING (\d+)", text).group(1)) == dbg.PENDING


def _c_layout(tmp_path, structs):
    """sizeof and field offsets of header structs, from a C program that
    includes dbg.h, built with gcc."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dbg.h"', "int main(void) {"]
    for cname, py in structs:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for field, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, field, cname, field))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {a: int(b) for a, b in (line.split() for line in out.splitlines())}


def test_struct_layouts_match_header(tmp_path):
    structs = [("dbg_config", dbg.Config), ("dbg_stats", dbg.Stats), ("dbg_input", dbg.Input),
               ("dbg_server_config", dbg.ServerConfig), ("dbg_server_stats", dbg.ServerStats),
               ("dbg_tuning", dbg.Tuning), ("dbg_probe_stats", dbg.ProbeStats)]
    got = _c_layout(tmp_path, structs)
    for cname, py in structs:
        assert got[cname] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got["%s.%s" % (cname, field)] == getattr(py, field).offset, (cname, field)


def test_strerror_and_config_init():
    L = dbg.lib()
    for code in range(0, -11, -1):
        assert L.dbg_strerror(code)
    assert L.dbg_strerror(-99) == b"unknown error"
    cfg = dbg.Config()
    cfg.flags = 7
    L.dbg_config_init(ctypes.byref(cfg))
    assert cfg.flags == 0 and cfg.device == -1 and cfg.load_factor == 0.0


def test_host_side_argument_errors_need_no_device():
    L = dbg.lib()
    h = ctypes.c_void_p()
    assert L.dbg_create(None, None) == dbg.E_INVAL
    cfg = dbg.Config()
    L.dbg_config_init(ctypes.byref(cfg))
    for lf in (-0.5, 1.0, 2.0):
        cfg.load_factor = lf
        assert L.dbg_create(ctypes.byref(cfg), ctypes.byref(h)) == dbg.E_INVAL
    cfg.flags = dbg.F_BINNED  # a binned table's segments overflow above the bound
    for lf in (0.86, 0.9):
        cfg.load_factor = lf
        assert L.dbg_create(ctypes.byref(cfg), ctypes.byref(h)) == dbg.E_INVAL
    text = open(os.path.join(ROOT, "include", "dbg.h")).read()
    assert float(re.search(r"#define DBG_BINNED_MAX_LOAD ([0-9.]+)", text).group(1)) == dbg.BINNED_MAX_LOAD
    cfg.flags = 0
    cfg.load_factor = 0.5
    cfg.block_size = 100  # not a multiple of 64
    assert L.dbg_create(ctypes.byref(cfg), ctypes.byref(h)) == dbg.E_INVAL
    assert L.dbg_build(None, None, None, 1, 21) == dbg.E_INVAL
    assert L.dbg_build_device(None, None, 0, None, 1, 21, None) == dbg.E_INVAL
    assert L.dbg_build_device_static(None, None, 0, None, 1, 21, None) == dbg.E_INVAL
    assert L.dbg_sync(None) == dbg.E_INVAL
    assert L.dbg_reset(None) == dbg.E_INVAL
    assert L.dbg_get_stats(None, None) == dbg.E_INVAL
    assert L.dbg_get_probe_stats(None, None) == dbg.E_INVAL
    n = ctypes.c_uint64()
    assert L.dbg_extract(None, None, None, 0, ctypes.byref(n)) == dbg.E_INVAL
    assert L.dbg_build_extract_device(None, None, 0, None, 1, 21, None, None, 0, ctypes.byref(n),
                                      None) == dbg.E_INVAL
    L.dbg_destroy(None)
    assert L.dbg_build_batch(None, None, 0, None, None) == dbg.OK
    assert L.dbg_build_batch(None, None, 2, None, None) == dbg.E_INVAL
    assert L.dbg_build_batch_device(None, 0, None, None, None, 0, None, None, None) == dbg.OK
    ms = ctypes.c_double()
    assert L.dbg_atomic_roofline(-1, 9, 1 << 20, 10, 256, 1, ctypes.byref(ms)) == dbg.E_INVAL
    assert L.dbg_atomic_roofline(-1, 0, 1 << 20, 10, 100, 1, ctypes.byref(ms)) == dbg.E_INVAL
    # server: configuration and handle checks come before any device call
    sc = dbg.ServerConfig()
    assert L.dbg_server_create(ctypes.byref(sc), None) == dbg.E_INVAL
    for lf in (-0.5, 1.0):
        sc.load_factor = lf
        assert L.dbg_server_create(ctypes.byref(sc), ctypes.byref(h)) == dbg.E_INVAL
    sc.load_factor, sc.slots = 0.5, 9
    assert L.dbg_server_create(ctypes.byref(sc), ctypes.byref(h)) == dbg.E_INVAL
    sc.load_factor, sc.slots = 0.9, 0  # binned by default: above the bound
    assert L.dbg_server_create(ctypes.byref(sc), ctypes.byref(h)) == dbg.E_INVAL
    rid = ctypes.c_uint64()
    st = ctypes.c_int32()
    assert L.dbg_server_submit(None, None, None, 0, 21, 0, ctypes.byref(rid)) == dbg.E_INVAL
    assert L.dbg_server_submit_device(None, None, 0, None, 0, 21, 0, ctypes.byref(rid)) == dbg.E_INVAL
    assert L.dbg_server_poll(None, 1, ctypes.byref(st)) == dbg.E_INVAL
    assert L.dbg_server_wait(None, 1, 0.0, ctypes.byref(st)) == dbg.E_INVAL
    assert L.dbg_server_release(None, 1) == dbg.E_INVAL
    assert L.dbg_server_get_stats(None, None) == dbg.E_INVAL
    L.dbg_server_destroy(None)
    n64 = ctypes.c_uint64()
    assert L.dbg_extract_normalized(None, 1, 0, None, None, 0, ctypes.byref(n64)) == dbg.E_INVAL
    assert L.dbg_contigs(None, None, 0, None, 0, ctypes.byref(n64), ctypes.byref(n64)) == dbg.E_INVAL
    assert L.dbg_contigs_device(None, None, 0, None, 0, ctypes.byref(n64), ctypes.byref(n64), None) == dbg.E_INVAL
    t = dbg.Tuning()
    assert L.dbg_autotune(-1, 0, None, None, None, None, 0, None, 0, 0, 0, ctypes.byref(t)) == dbg.E_INVAL
    rb = (ctypes.c_uint64 * 3)(0, 1, 1)
    ks = (ctypes.c_uint32 * 2)(65, 21)
    off = (ctypes.c_uint64 * 2)(0, 0)
    assert L.dbg_autotune(-1, 1, rb, ks, None, None, 0, off, 0, 0, 0, ctypes.byref(t)) == dbg.E_INVAL
    ks[0] = 33  # long k only for a single graph
    assert L.dbg_autotune(-1, 2, rb, ks, None, None, 0, off, 0, 0, 0, ctypes.byref(t)) == dbg.E_INVAL
    cfg = dbg.Config()
    L.dbg_config_init(ctypes.byref(cfg))
    cfg.flags = dbg.F_GRAPH | dbg.F_MERGE
    t.load_factor, t.flags, t.block_size, t.windows_per_thread = 0.6, dbg.F_BINNED, 0, 0
    t.bin_chunks, t.bin_scatter_div, t.bin_shape1, t.bin_shape2 = 32, 2, dbg.SHAPE_BIG, dbg.SHAPE_STAGED
    L.dbg_config_apply_tuning(ctypes.byref(cfg), ctypes.byref(t))
    assert cfg.flags == dbg.F_GRAPH | dbg.F_BINNED and cfg.load_factor == 0.6
    assert cfg.bin_chunks == 32 and cfg.bin_scatter_div == 2
    assert (cfg.bin_shape1, cfg.bin_shape2) == (dbg.SHAPE_BIG, dbg.SHAPE_STAGED)
    cfg.bin_chunks = 1 << 20  # more chunks per workgroup than a pass has
    assert L.dbg_create(ctypes.byref(cfg), ctypes.byref(h)) == dbg.E_INVAL
    cfg.bin_chunks, cfg.bin_shape1, cfg.bin_shape2 = 0, 5, 0  # shapes are 0 (automatic) to 4 (wide big tiles)
    assert L.dbg_create(ctypes.byref(cfg), ctypes.byref(h)) == dbg.E_INVAL
    cfg.bin_shape1, cfg.bin_shape2 = 0, 5
    assert L.dbg_create(ctypes.byref(cfg), ctypes.byref(h)) == dbg.E_INVAL
    # the search space: binned load factors x chunks x scatter shape pairs x divisors, direct load factors x
    # shapes x merging
    nb = len(dbg.autotune_space(True))
    nd = len(dbg.autotune_space(False))
    assert nb == 4 * 5 * 6 * 4 and nd == 4 * 3 * 3 * 2
    assert all(c.flags == dbg.F_BINNED and 0 < c.load_factor < dbg.BINNED_MAX_LOAD for c in dbg.autotune_space(True))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(dbg, "_lib", None)
    monkeypatch.setattr(dbg, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="not built"):
        dbg.lib()


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2401_02756_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                for pat in (r"^\s*import oracle", r"^\s*from oracle", r"liboracle", r"dbg_oracle"):
                    assert not re.search(pat, text, flags=re.M), (f, pat)
