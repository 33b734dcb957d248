"""CPU oracle for the A-Bruijn graph build -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it,
and it shares no code with the GPU path: its C core (``dbg_oracle.c``) packs,
hashes and counts on its own.

Contents:
  * ``build_graph``   -- the graph as sorted records (the C core, the plain
                         definition of the build; see ``dbg_oracle.c``);
  * ``vertex_counts`` -- one vertex's four counters by scanning every window;
  * ``brute``         -- a second, string-based brute force for tiny inputs;
  * ``invariants``    -- properties any correct graph satisfies;
  * ``euler``         -- Eulerian path over the graph's edge multiplicities.

Output form (the canonical comparison form): ``keys`` is ``uint64[V]``
ascending, ``counts`` is ``uint32[V, 4]`` with column c the counter of letter
code c (A=0, C=1, T=2, G=3).  A key is the (k-1)-mer as 2-bit codes, first
base most significant.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dbg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_LFDBG_SRC = os.path.join(_HERE, "lfdbg_cpu.cpp")
_LFDBG_PATH = os.path.join(_HERE, "_liblfdbg.so")

OK, E_INVAL, E_K, E_BASE, E_NOMEM = 0, -1, -2, -3, -4

# Letter code of the paper: counter index (c >> 1) & 3.
LETTERS = "ACTG"

_lib = None


def compile_oracle(force: bool = False) -> str:
    """Compile the C core with gcc into ``oracle/_liboracle.so`` (and the
    CPU baseline of the paper's threaded build into ``oracle/_liblfdbg.so``)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    if force or not os.path.exists(_LFDBG_PATH):
        tmp = _LFDBG_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-Wextra", "-pthread", "-shared",
                               "-fPIC", "-o", tmp, _LFDBG_SRC])
        os.replace(tmp, _LFDBG_PATH)
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            compile_oracle()
        L = ctypes.CDLL(_LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.POINTER(u64p), ctypes.POINTER(u32p),
                                   ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_build.restype = ctypes.c_int
        L.oracle_validate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_uint32]
        L.oracle_validate.restype = ctypes.c_int
        L.oracle_vertex_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint64, u32p]
        L.oracle_vertex_counts.restype = ctypes.c_int
        L.oracle_partition_many.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                            ctypes.c_void_p]
        L.oracle_partition_many.restype = None
        L.oracle_contigs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_contigs.restype = ctypes.c_int
        L.oracle_strings_digest.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]
        L.oracle_strings_digest.restype = ctypes.c_uint64
        L.oracle_normalize.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_normalize.restype = None
        L.oracle_build_wide.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64)]
        L.oracle_build_wide.restype = ctypes.c_int
        L.oracle_free.argtypes = [ctypes.c_void_p]
        L.oracle_free.restype = None
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error %d" % code)
        self.code = code


def _as_inputs(reads, offsets):
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    return reads, offsets


def validate(reads, offsets, k: int) -> int:
    reads, offsets = _as_inputs(reads, offsets)
    n = max(0, offsets.shape[0] - 1)
    return int(lib().oracle_validate(reads.ctypes.data if reads.size else None,
                                     offsets.ctypes.data if offsets.size else None,
                                     n, int(k)))


def build_graph(reads, offsets, k: int, part_count: int = 1, part_index: int = 0):
    """Graph of the reads as ``(keys uint64[V] ascending, counts uint32[V, 4])``."""
    reads, offsets = _as_inputs(reads, offsets)
    n = max(0, offsets.shape[0] - 1)
    pk = ctypes.POINTER(ctypes.c_uint64)()
    pc = ctypes.POINTER(ctypes.c_uint32)()
    nv = ctypes.c_uint64(0)
    rc = lib().oracle_build(reads.ctypes.data if reads.size else None,
                            offsets.ctypes.data if offsets.size else None,
                            n, int(k), int(part_count), int(part_index),
                            ctypes.byref(pk), ctypes.byref(pc), ctypes.byref(nv))
    if rc != OK:
        raise OracleError(rc)
    V = int(nv.value)
    try:
        keys = np.ctypeslib.as_array(pk, shape=(V,)).copy() if V else np.zeros(0, np.uint64)
        counts = (np.ctypeslib.as_array(pc, shape=(V * 4,)).copy().reshape(V, 4)
                  if V else np.zeros((0, 4), np.uint32))
    finally:
        lib().oracle_free(ctypes.cast(pk, ctypes.c_void_p))
        lib().oracle_free(ctypes.cast(pc, ctypes.c_void_p))
    return keys, counts


def build_graph_parallel(reads, offsets, k: int, threads: int = 0):
    """Same result as ``build_graph``, computed as ``threads`` key-space
    partitions in parallel threads (the C core releases the GIL) and merged.
    Each partition is an exact slice of the graph, so the union is exact."""
    import concurrent.futures

    P = threads or min(16, os.cpu_count() or 1)
    if P <= 1:
        return build_graph(reads, offsets, k)
    reads, offsets = _as_inputs(reads, offsets)
    with concurrent.futures.ThreadPoolExecutor(P) as ex:
        parts = list(ex.map(lambda p: build_graph(reads, offsets, k, P, p), range(P)))
    keys = np.concatenate([p[0] for p in parts])
    counts = np.concatenate([p[1] for p in parts])
    order = np.argsort(keys, kind="stable")
    return keys[order], counts[order]


def build_graph_chunked(reads, offsets, k: int, part_count: int = 1, part_index: int = 0,
                        chunks: int = 0):
    """Same result as ``build_graph(reads, offsets, k, part_count, part_index)``,
    computed over ``chunks`` contiguous read ranges in parallel threads and
    merged.  Exact because the graph is a multiset count over reads: the
    vertex set of the whole is the union of the ranges' vertex sets and each
    counter is the sum of the ranges' counters."""
    import concurrent.futures

    reads, offsets = _as_inputs(reads, offsets)
    n = max(0, offsets.shape[0] - 1)
    C = max(1, min(chunks or min(16, os.cpu_count() or 1), n))
    if C == 1:
        return build_graph(reads, offsets, k, part_count, part_index)
    cuts = [n * c // C for c in range(C + 1)]
    with concurrent.futures.ThreadPoolExecutor(C) as ex:
        parts = list(ex.map(lambda c: build_graph(reads, offsets[cuts[c]:cuts[c + 1] + 1], k,
                                                  part_count, part_index), range(C)))
    keys = np.concatenate([p[0] for p in parts])
    counts = np.concatenate([p[1] for p in parts]).astype(np.uint64)
    order = np.argsort(keys, kind="stable")
    keys, counts = keys[order], counts[order]
    uniq, first = np.unique(keys, return_index=True)
    summed = np.add.reduceat(counts, first, axis=0) if keys.size else counts
    return uniq, summed.astype(np.uint32)


def contigs(keys, counts, k: int):
    """Contigs of the graph ``(keys ascending, counts[V, 4])`` as the paper's
    findContigs defines them (see ``oracle_contigs``): ``(seq uint8[],
    offsets uint64[n + 1])``, contig i being ``seq[offsets[i]:offsets[i+1]]``."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    n = keys.shape[0]
    ps, po = ctypes.c_void_p(), ctypes.c_void_p()
    nc, sl = ctypes.c_uint64(0), ctypes.c_uint64(0)
    rc = lib().oracle_contigs(keys.ctypes.data if n else None, counts.ctypes.data if n else None, n, int(k),
                              ctypes.byref(ps), ctypes.byref(po), ctypes.byref(nc), ctypes.byref(sl))
    if rc != OK:
        raise OracleError(rc)
    try:
        seq = (np.ctypeslib.as_array(ctypes.cast(ps, ctypes.POINTER(ctypes.c_uint8)), shape=(sl.value,)).copy()
               if sl.value else np.zeros(0, np.uint8))
        off = np.ctypeslib.as_array(ctypes.cast(po, ctypes.POINTER(ctypes.c_uint64)), shape=(nc.value + 1,)).copy()
    finally:
        lib().oracle_free(ps)
        lib().oracle_free(po)
    return seq, off


def contig_strings(seq, off) -> list:
    """The contigs as a sorted list of bytes (for small sets)."""
    seq = np.asarray(seq, dtype=np.uint8)
    return sorted(seq[off[i]:off[i + 1]].tobytes() for i in range(len(off) - 1))


def strings_digest(seq, off) -> int:
    """Order-free 64-bit digest of a set of strings (``oracle_strings_digest``)."""
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    return int(lib().oracle_strings_digest(seq.ctypes.data if seq.size else None, off.ctypes.data,
                                           off.shape[0] - 1))


def normalize(counts, genome_size: int, total_kmers: int):
    """Normalized counters (``oracle_normalize``): (uint32 array, uint8 array
    saturated at 255) of the same shape as ``counts``."""
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    o32 = np.empty_like(c)
    o8 = np.empty(c.shape, dtype=np.uint8)
    if c.size:
        lib().oracle_normalize(c.ctypes.data, c.size, int(genome_size), int(total_kmers), o32.ctypes.data,
                               o8.ctypes.data)
    return o32, o8


_lfdbg = None


def lfdbg_build(reads, offsets, k: int, threads: int, buckets: int = 0):
    """The paper's lock-free build on CPU threads (``oracle/lfdbg_cpu.cpp``):
    ``(keys ascending, counts[V, 4], seconds of the threaded build)``.
    ``buckets`` is the paper's table size (default: the number of windows)."""
    global _lfdbg
    if _lfdbg is None:
        if not os.path.exists(_LFDBG_PATH):
            compile_oracle()
        L = ctypes.CDLL(_LFDBG_PATH)
        L.lfdbg_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_double)]
        L.lfdbg_build.restype = ctypes.c_int
        L.lfdbg_free.argtypes = [ctypes.c_void_p]
        L.lfdbg_free.restype = None
        _lfdbg = L
    reads, offsets = _as_inputs(reads, offsets)
    n = max(0, offsets.shape[0] - 1)
    if not buckets:
        buckets = max(1, int(np.maximum(np.diff(offsets.astype(np.int64)) - k + 2, 0).sum()))
    pk, pc = ctypes.c_void_p(), ctypes.c_void_p()
    nv, sec = ctypes.c_uint64(0), ctypes.c_double(0)
    rc = _lfdbg.lfdbg_build(reads.ctypes.data if reads.size else None, offsets.ctypes.data if offsets.size else None,
                            n, int(k), int(threads), int(buckets), ctypes.byref(pk), ctypes.byref(pc),
                            ctypes.byref(nv), ctypes.byref(sec))
    if rc != 0:
        raise OracleError(rc)
    V = int(nv.value)
    try:
        keys = (np.ctypeslib.as_array(ctypes.cast(pk, ctypes.POINTER(ctypes.c_uint64)), shape=(V,)).copy()
                if V else np.zeros(0, np.uint64))
        counts = (np.ctypeslib.as_array(ctypes.cast(pc, ctypes.POINTER(ctypes.c_uint32)), shape=(V * 4,))
                  .copy().reshape(V, 4) if V else np.zeros((0, 4), np.uint32))
    finally:
        _lfdbg.lfdbg_free(pk)
        _lfdbg.lfdbg_free(pc)
    return keys, counts, float(sec.value)


def build_graph_wide(reads, offsets, k: int):
    """Graph for 2 <= k <= 64: ``(hi uint64[V], lo uint64[V], counts[V, 4])``
    sorted by (hi, lo); the (k-1)-mer key is hi * 2^64 + lo."""
    reads, offsets = _as_inputs(reads, offsets)
    n = max(0, offsets.shape[0] - 1)
    ph, pl, pc = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    nv = ctypes.c_uint64(0)
    rc = lib().oracle_build_wide(reads.ctypes.data if reads.size else None,
                                 offsets.ctypes.data if offsets.size else None, n, int(k),
                                 ctypes.byref(ph), ctypes.byref(pl), ctypes.byref(pc), ctypes.byref(nv))
    if rc != OK:
        raise OracleError(rc)
    V = int(nv.value)
    u64p, u32p = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)
    try:
        hi = np.ctypeslib.as_array(ctypes.cast(ph, u64p), shape=(V,)).copy() if V else np.zeros(0, np.uint64)
        lo = np.ctypeslib.as_array(ctypes.cast(pl, u64p), shape=(V,)).copy() if V else np.zeros(0, np.uint64)
        counts = (np.ctypeslib.as_array(ctypes.cast(pc, u32p), shape=(V * 4,)).copy().reshape(V, 4)
                  if V else np.zeros((0, 4), np.uint32))
    finally:
        for p in (ph, pl, pc):
            lib().oracle_free(p)
    return hi, lo, counts


def decode_wide_key(hi: int, lo: int, k: int) -> str:
    """The (k-1)-mer string of a two-word key."""
    v = (int(hi) << 64) | int(lo)
    return "".join("ACTG"[(v >> (2 * (k - 2 - i))) & 3] for i in range(k - 1))


def vertex_counts(reads, offsets, k: int, key: int):
    """(present, counts[4]) of one vertex by scanning every window."""
    reads, offsets = _as_inputs(reads, offsets)
    n = max(0, offsets.shape[0] - 1)
    out = (ctypes.c_uint32 * 4)()
    seen = lib().oracle_vertex_counts(reads.ctypes.data if reads.size else None,
                                      offsets.ctypes.data if offsets.size else None,
                                      n, int(k), int(key), out)
    return bool(seen), np.array(list(out), dtype=np.uint32)


def partition_of(keys, part_count: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    parts = np.empty(keys.shape[0], dtype=np.uint32)
    if keys.size:
        lib().oracle_partition_many(keys.ctypes.data, keys.shape[0], int(part_count),
                                    parts.ctypes.data)
    return parts


def decode_key(key: int, k: int) -> str:
    """(k-1)-mer string of a key (first base in the most significant bits)."""
    n = k - 1
    return "".join(LETTERS[(int(key) >> (2 * (n - 1 - i))) & 3] for i in range(n))


def graph_to_dict(keys, counts, k: int) -> dict:
    """{vertex string: {letter: count}} with zero counters omitted."""
    out = {}
    for key, c in zip(keys.tolist(), counts.tolist()):
        out[decode_key(key, k)] = {LETTERS[i]: int(c[i]) for i in range(4) if c[i]}
    return out
