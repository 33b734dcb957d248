"""Exact comparison of a graph's records with the oracle's, without sorting
the graph's records (tests/host/record_compare.c, built here with gcc; the C
call releases the GIL, so partitions or read sets compare in parallel
threads)."""

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "record_compare.c")
LIB = os.path.join(HERE, "host", "_librecord_compare.so")


class Result(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in
                ("selected", "missing", "wrong", "repeated", "found", "first_bad")]


_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                tmp = LIB + ".tmp%d" % os.getpid()
                subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, SRC])
                os.replace(tmp, LIB)
            L = ctypes.CDLL(LIB)
            L.cmp_records.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.POINTER(Result)]
            L.cmp_records.restype = ctypes.c_int
            _lib = L
    return _lib


def compare(want, got, part=None, p=0) -> dict:
    """Compare oracle records ``want = (keys, counts[V, 4])`` (one key-space
    partition) with graph records ``got`` in any order, restricted to
    ``part == p`` when ``part`` is given."""
    wk = np.ascontiguousarray(want[0], dtype=np.uint64)
    wc = np.ascontiguousarray(want[1], dtype=np.uint32)
    gk = np.ascontiguousarray(got[0], dtype=np.uint64)
    gc = np.ascontiguousarray(got[1], dtype=np.uint32)
    assert wc.shape == (wk.shape[0], 4) and gc.shape == (gk.shape[0], 4)
    if part is not None:
        part = np.ascontiguousarray(part, dtype=np.uint32)
        assert part.shape[0] == gk.shape[0]
    r = Result()
    rc = lib().cmp_records(wk.ctypes.data if wk.size else None, wc.ctypes.data if wc.size else None, wk.shape[0],
                           gk.ctypes.data if gk.size else None, gc.ctypes.data if gc.size else None, gk.shape[0],
                           part.ctypes.data if part is not None and part.size else None, int(p), ctypes.byref(r))
    assert rc == 0, "record comparison could not allocate its index"
    out = {name: int(getattr(r, name)) for name, _ in Result._fields_}
    out["oracle"] = int(wk.shape[0])
    return out


def exact(res: dict) -> bool:
    return (res["missing"] == 0 and res["wrong"] == 0 and res["repeated"] == 0 and
            res["found"] == res["oracle"] and res["selected"] == res["oracle"])


def assert_exact(want, got, what, part=None, p=0) -> dict:
    res = compare(want, got, part, p)
    assert exact(res), "%s: %s" % (what, res)
    return res
