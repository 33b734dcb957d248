"""Python binding of libdbg, the MI355X A-Bruijn graph builder.

Argument marshalling only: every step of the build runs in the HIP kernels of
``libdbg.so`` (``csrc/``), called through its C ABI (``include/dbg.h``).
There is no CPU fallback: if the library is not built, every entry point
raises.  PyTorch is used only to hand device buffers and streams to the
library (``build_device``/``extract_device``/``build_batch_device``).

Conventions (the same as the C ABI): read i is
``reads[offsets[i]:offsets[i+1]]``; keys are (k-1)-mers as 2-bit letter codes
(A=0, C=1, T=2, G=3), first base most significant; ``counts[:, c]`` is the
counter of letter code c.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libdbg.so")

OK = 0
PENDING = 1
E_INVAL, E_K, E_BASE, E_NOMEM, E_FULL, E_SPACE, E_DEVICE, E_RANGE, E_STATE, E_SCRATCH = range(-1, -11, -1)
F_MERGE, F_TIMING, F_ENTRY32, F_BINNED, F_GRAPH, F_STATS, F_TEST_HASH = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40

# every symbol include/dbg.h declares
EXPORTS = (
    "dbg_config_init", "dbg_create", "dbg_build", "dbg_build_device", "dbg_sync",
    "dbg_extract", "dbg_extract_device", "dbg_reset", "dbg_get_stats", "dbg_destroy",
    "dbg_strerror", "dbg_build_batch", "dbg_build_batch_device", "dbg_atomic_roofline",
    "dbg_get_phase_times", "dbg_server_create", "dbg_server_submit", "dbg_server_submit_device",
    "dbg_server_poll", "dbg_server_wait", "dbg_server_graph", "dbg_server_times",
    "dbg_server_release", "dbg_server_get_stats", "dbg_server_destroy", "dbg_autotune",
    "dbg_config_apply_tuning", "dbg_contigs", "dbg_contigs_device", "dbg_extract_normalized",
    "dbg_build_extract_device", "dbg_build_device_static", "dbg_get_probe_stats", "dbg_autotune_space",
)
NORM_U8 = 0x1
BINNED_MAX_LOAD = 0.85  # DBG_BINNED_MAX_LOAD: the largest load factor dbg_create takes for a binned graph
# phases of a timed binned build launched without graphs (dbg_get_phase_times)
BINNED_PHASES = ("setup", "plan", "count1", "scan1", "scatter1", "plan2", "count2", "scan2", "scatter2",
                 "starts", "reduce")
TUNE_FORCE = 0x1
# partition scatter shapes (dbg_config bin_shape1 / bin_shape2)
SHAPE_AUTO, SHAPE_TILES, SHAPE_STAGED, SHAPE_BIG, SHAPE_BIG_WIDE = 0, 1, 2, 3, 4


class Config(ctypes.Structure):
    _fields_ = [
        ("expected_vertices", ctypes.c_uint64),
        ("capacity", ctypes.c_uint64),
        ("load_factor", ctypes.c_double),
        ("device", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("block_size", ctypes.c_uint32),
        ("windows_per_thread", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
        ("bin_chunks", ctypes.c_uint32),
        ("bin_scatter_div", ctypes.c_uint32),
        ("bin_shape1", ctypes.c_uint32),
        ("bin_shape2", ctypes.c_uint32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("capacity", ctypes.c_uint64),
        ("table_bytes", ctypes.c_uint64),
        ("vertices", ctypes.c_uint64),
        ("inserts", ctypes.c_uint64),
        ("windows", ctypes.c_uint64),
        ("builds", ctypes.c_uint64),
        ("k", ctypes.c_uint32),
        ("status", ctypes.c_int32),
        ("last_build_ms", ctypes.c_double),
        ("last_total_ms", ctypes.c_double),
        ("block_size", ctypes.c_uint32),
        ("windows_per_thread", ctypes.c_uint32),
        ("grid_size", ctypes.c_uint32),
        ("entry_bytes", ctypes.c_uint32),
        ("graph_captures", ctypes.c_uint64),
        ("graph_replays", ctypes.c_uint64),
        ("binned", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
        ("bin_chunks", ctypes.c_uint32),
        ("bin_scatter_div", ctypes.c_uint32),
        ("bin_shape1", ctypes.c_uint32),
        ("bin_shape2", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ProbeStats(ctypes.Structure):
    _fields_ = [("lookups", ctypes.c_uint64), ("probes", ctypes.c_uint64), ("cas_attempts", ctypes.c_uint64),
                ("cas_lost", ctypes.c_uint64), ("probe_hist", ctypes.c_uint64 * 8)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "probe_hist"}
        d["probe_hist"] = [int(x) for x in self.probe_hist]
        return d


class Input(ctypes.Structure):
    _fields_ = [
        ("reads", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p),
        ("n_reads", ctypes.c_uint64),
        ("k", ctypes.c_uint32),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_uint64),
        ("max_batch_bytes", ctypes.c_uint64),
        ("max_batch", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("load_factor", ctypes.c_double),
        ("device", ctypes.c_int32),
        ("slots", ctypes.c_uint32),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "submitted", "admitted", "completed", "released", "rejected", "queued", "running",
        "resident_bytes", "passes", "max_in_flight")]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [
        ("load_factor", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("block_size", ctypes.c_uint32),
        ("windows_per_thread", ctypes.c_uint32),
        ("candidates", ctypes.c_uint32),
        ("best_ms", ctypes.c_double),
        ("default_ms", ctypes.c_double),
        ("from_cache", ctypes.c_uint32),
        ("bin_chunks", ctypes.c_uint32),
        ("bin_scatter_div", ctypes.c_uint32),
        ("bin_shape1", ctypes.c_uint32),
        ("bin_shape2", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}

    def graph_kwargs(self) -> dict:
        """Keyword arguments of ``Graph`` that apply this tuning."""
        return dict(load_factor=self.load_factor, block_size=self.block_size,
                    windows_per_thread=self.windows_per_thread, flags=self.flags,
                    bin_chunks=self.bin_chunks, bin_scatter_div=self.bin_scatter_div,
                    bin_shape1=self.bin_shape1, bin_shape2=self.bin_shape2)


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded ``libdbg.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdbg.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
        sig = {
            "dbg_config_init": (None, [ctypes.POINTER(Config)]),
            "dbg_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(vp)]),
            "dbg_build": (ctypes.c_int, [vp, vp, vp, u64, u32]),
            "dbg_build_device": (ctypes.c_int, [vp, vp, u64, vp, u64, u32, vp]),
            "dbg_build_device_static": (ctypes.c_int, [vp, vp, u64, vp, u64, u32, vp]),
            "dbg_sync": (ctypes.c_int, [vp]),
            "dbg_extract": (ctypes.c_int, [vp, vp, vp, u64, ctypes.POINTER(u64)]),
            "dbg_extract_device": (ctypes.c_int, [vp, vp, vp, u64, ctypes.POINTER(u64), vp]),
            "dbg_build_extract_device": (ctypes.c_int, [vp, vp, u64, vp, u64, u32, vp, vp, u64,
                                                        ctypes.POINTER(u64), vp]),
            "dbg_reset": (ctypes.c_int, [vp]),
            "dbg_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(Stats)]),
            "dbg_get_probe_stats": (ctypes.c_int, [vp, ctypes.POINTER(ProbeStats)]),
            "dbg_destroy": (None, [vp]),
            "dbg_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "dbg_build_batch": (ctypes.c_int, [vp, vp, u32, vp, vp]),
            "dbg_build_batch_device": (ctypes.c_int, [vp, u32, vp, vp, vp, u64, vp, vp, vp]),
            "dbg_atomic_roofline": (ctypes.c_int, [i32, u32, u64, u64, u32, u32,
                                                   ctypes.POINTER(ctypes.c_double)]),
            "dbg_get_phase_times": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), u32,
                                                   ctypes.POINTER(u32)]),
            "dbg_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
            "dbg_server_submit": (ctypes.c_int, [vp, vp, vp, u64, u32, u64, ctypes.POINTER(u64)]),
            "dbg_server_submit_device": (ctypes.c_int, [vp, vp, u64, vp, u64, u32, u64,
                                                        ctypes.POINTER(u64)]),
            "dbg_server_poll": (ctypes.c_int, [vp, u64, ctypes.POINTER(i32)]),
            "dbg_server_wait": (ctypes.c_int, [vp, u64, ctypes.c_double, ctypes.POINTER(i32)]),
            "dbg_server_graph": (ctypes.c_int, [vp, u64, ctypes.POINTER(vp)]),
            "dbg_server_times": (ctypes.c_int, [vp, u64, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double)]),
            "dbg_server_release": (ctypes.c_int, [vp, u64]),
            "dbg_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
            "dbg_server_destroy": (None, [vp]),
            "dbg_autotune": (ctypes.c_int, [i32, u32, vp, vp, vp, vp, u64, vp, u32, u32, u32,
                                            ctypes.POINTER(Tuning)]),
            "dbg_config_apply_tuning": (None, [ctypes.POINTER(Config), ctypes.POINTER(Tuning)]),
            "dbg_autotune_space": (ctypes.c_int, [u32, ctypes.POINTER(Tuning), u32, ctypes.POINTER(u32)]),
            "dbg_extract_normalized": (ctypes.c_int, [vp, u64, u32, vp, vp, u64, ctypes.POINTER(u64)]),
            "dbg_contigs": (ctypes.c_int, [vp, vp, u64, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
            "dbg_contigs_device": (ctypes.c_int, [vp, vp, u64, vp, u64, ctypes.POINTER(u64),
                                                  ctypes.POINTER(u64), vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DbgError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        msg = lib().dbg_strerror(code).decode()
        super().__init__("%s%s (%d)" % (where + ": " if where else "", msg, code))
        self.code = code


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise DbgError(rc, where)


def _host_inputs(reads, offsets):
    if isinstance(reads, (bytes, bytearray)):
        reads = np.frombuffer(bytes(reads), dtype=np.uint8)
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    return reads, offsets


def _ptr(t) -> int:
    """Device pointer of a torch tensor (or an int)."""
    return int(t) if isinstance(t, int) else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Graph:
    """One graph handle (``dbg_create`` .. ``dbg_destroy``)."""

    def __init__(self, expected_vertices: int = 0, capacity: int = 0, load_factor: float = 0.0,
                 device: int = -1, flags: int = 0, block_size: int = 0,
                 windows_per_thread: int = 0, stream=None, bin_chunks: int = 0, bin_scatter_div: int = 0,
                 bin_shape1: int = 0, bin_shape2: int = 0, _borrowed=None):
        self._owned = _borrowed is None
        if not self._owned:
            self._h = ctypes.c_void_p(_borrowed)
            return
        cfg = Config()
        lib().dbg_config_init(ctypes.byref(cfg))
        cfg.expected_vertices = int(expected_vertices)
        cfg.capacity = int(capacity)
        cfg.load_factor = float(load_factor)
        cfg.device = int(device)
        cfg.flags = int(flags)
        cfg.block_size = int(block_size)
        cfg.windows_per_thread = int(windows_per_thread)
        cfg.stream = _stream(stream)
        cfg.bin_chunks = int(bin_chunks)
        cfg.bin_scatter_div = int(bin_scatter_div)
        cfg.bin_shape1 = int(bin_shape1)
        cfg.bin_shape2 = int(bin_shape2)
        h = ctypes.c_void_p()
        _check(lib().dbg_create(ctypes.byref(cfg), ctypes.byref(h)), "dbg_create")
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("graph is closed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            if getattr(self, "_owned", True):
                lib().dbg_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def build(self, reads, offsets, k: int) -> None:
        reads, offsets = _host_inputs(reads, offsets)
        n = max(0, offsets.shape[0] - 1)
        rc = lib().dbg_build(self.handle, reads.ctypes.data if reads.size else None,
                             offsets.ctypes.data if offsets.size else None, n, int(k))
        _check(rc, "dbg_build")

    def build_device(self, d_reads, d_offsets, k: int, n_reads: int | None = None,
                     reads_len: int | None = None, stream=None) -> None:
        """Enqueue a build from device tensors (uint8 reads, int64/uint64 offsets)."""
        n = int(d_offsets.numel() - 1) if n_reads is None else int(n_reads)
        ln = int(d_reads.numel()) if reads_len is None else int(reads_len)
        rc = lib().dbg_build_device(self.handle, _ptr(d_reads), ln, _ptr(d_offsets), n, int(k),
                                    _stream(stream))
        _check(rc, "dbg_build_device")

    def build_device_static(self, d_reads, d_offsets, k: int, n_reads: int | None = None,
                            reads_len: int | None = None, stream=None) -> None:
        """``dbg_build_device_static``: the device build with its scratch in
        the library's static device array (no allocation; synchronous)."""
        n = int(d_offsets.numel() - 1) if n_reads is None else int(n_reads)
        ln = int(d_reads.numel()) if reads_len is None else int(reads_len)
        rc = lib().dbg_build_device_static(self.handle, _ptr(d_reads), ln, _ptr(d_offsets), n, int(k),
                                           _stream(stream))
        _check(rc, "dbg_build_device_static")

    def build_extract_device(self, d_reads, d_offsets, k: int, d_keys, d_counts, n_reads: int | None = None,
                             reads_len: int | None = None, stream=None) -> int:
        """``dbg_build_extract_device``: build from device tensors, then write
        every vertex of the graph to d_keys / d_counts (device tensors, any
        order).  Returns the vertex count."""
        n = int(d_offsets.numel() - 1) if n_reads is None else int(n_reads)
        ln = int(d_reads.numel()) if reads_len is None else int(reads_len)
        kw = 2 if int(k) > 32 else 1
        v = ctypes.c_uint64(0)
        rc = lib().dbg_build_extract_device(self.handle, _ptr(d_reads), ln, _ptr(d_offsets), n, int(k),
                                            _ptr(d_keys) if d_keys is not None else None,
                                            _ptr(d_counts) if d_counts is not None else None,
                                            int(d_keys.numel()) // kw if d_keys is not None else 0,
                                            ctypes.byref(v), _stream(stream))
        _check(rc, "dbg_build_extract_device")
        return int(v.value)

    def sync(self) -> None:
        _check(lib().dbg_sync(self.handle), "dbg_sync")

    def vertex_count(self) -> int:
        n = ctypes.c_uint64(0)
        _check(lib().dbg_extract(self.handle, None, None, 0, ctypes.byref(n)), "dbg_extract")
        return int(n.value)

    def key_words(self) -> int:
        """uint64 words per extracted key: 2 for k > 32 (high word, low word)."""
        return 2 if self.stats()["k"] > 32 else 1

    def extract(self):
        """(keys uint64[V], counts uint32[V, 4]) in unspecified order; for
        k > 32 keys is uint64[V, 2] (high word, low word)."""
        V = self.vertex_count()
        keys = np.empty((V, 2) if self.key_words() == 2 else V, dtype=np.uint64)
        counts = np.empty((V, 4), dtype=np.uint32)
        n = ctypes.c_uint64(0)
        if V:
            rc = lib().dbg_extract(self.handle, keys.ctypes.data, counts.ctypes.data, V,
                                   ctypes.byref(n))
            _check(rc, "dbg_extract")
        return keys, counts

    def extract_sorted(self):
        keys, counts = self.extract()
        if keys.ndim == 2:
            order = np.lexsort((keys[:, 1], keys[:, 0]))
        else:
            order = np.argsort(keys, kind="stable")
        return keys[order], counts[order]

    def extract_device(self, d_keys, d_counts, stream=None) -> int:
        n = ctypes.c_uint64(0)
        rc = lib().dbg_extract_device(self.handle, _ptr(d_keys), _ptr(d_counts),
                                      int(d_keys.numel()) // self.key_words(), ctypes.byref(n), _stream(stream))
        _check(rc, "dbg_extract_device")
        return int(n.value)

    def extract_normalized(self, genome_size: int, u8: bool = False):
        """(keys uint64[V], counts[V, 4]) with every counter normalized by the
        expected k-mer duplication (dbg_extract_normalized); uint32 counts,
        or uint8 saturated at 255 with u8=True."""
        V = self.vertex_count()
        keys = np.empty((V, 2) if self.key_words() == 2 else V, dtype=np.uint64)
        counts = np.empty((V, 4), dtype=np.uint8 if u8 else np.uint32)
        n = ctypes.c_uint64(0)
        if V:
            rc = lib().dbg_extract_normalized(self.handle, int(genome_size), NORM_U8 if u8 else 0,
                                              keys.ctypes.data, counts.ctypes.data, V, ctypes.byref(n))
            _check(rc, "dbg_extract_normalized")
        return keys, counts

    def contig_sizes(self) -> tuple[int, int]:
        """(number of contigs, total bases) -- computes the contigs."""
        n, ln = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().dbg_contigs(self.handle, None, 0, None, 0, ctypes.byref(n), ctypes.byref(ln)),
               "dbg_contigs")
        return int(n.value), int(ln.value)

    def contigs(self):
        """(seq uint8[total], offsets uint64[n + 1]): contig i is seq[offsets[i]:offsets[i+1]]."""
        n, ln = self.contig_sizes()
        seq = np.empty(max(ln, 1), dtype=np.uint8)
        off = np.empty(n + 1, dtype=np.uint64)
        nn, ll = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().dbg_contigs(self.handle, seq.ctypes.data, seq.shape[0], off.ctypes.data, off.shape[0],
                                 ctypes.byref(nn), ctypes.byref(ll)), "dbg_contigs")
        return seq[:ln], off

    def contigs_device(self, d_seq, d_offsets, stream=None) -> tuple[int, int]:
        """Contigs into device tensors (uint8, int64/uint64); returns (n, total bases)."""
        n, ln = ctypes.c_uint64(0), ctypes.c_uint64(0)
        rc = lib().dbg_contigs_device(self.handle, _ptr(d_seq), int(d_seq.numel()), _ptr(d_offsets),
                                      int(d_offsets.numel()), ctypes.byref(n), ctypes.byref(ln), _stream(stream))
        _check(rc, "dbg_contigs_device")
        return int(n.value), int(ln.value)

    def phase_times(self) -> list[float]:
        """Per-phase device ms of the last timed build (see dbg_get_phase_times;
        binned builds launched without graphs: BINNED_PHASES)."""
        buf = (ctypes.c_double * 16)()
        n = ctypes.c_uint32(0)
        _check(lib().dbg_get_phase_times(self.handle, buf, 16, ctypes.byref(n)), "dbg_get_phase_times")
        return [float(buf[i]) for i in range(min(16, n.value))]

    def reset(self) -> None:
        _check(lib().dbg_reset(self.handle), "dbg_reset")

    def stats(self) -> dict:
        s = Stats()
        _check(lib().dbg_get_stats(self.handle, ctypes.byref(s)), "dbg_get_stats")
        return s.as_dict()

    def probe_stats(self) -> dict:
        """``dbg_get_probe_stats``: lookups, probes, compare-and-swaps and lost
        races of the graph's builds (zeros without F_STATS)."""
        s = ProbeStats()
        _check(lib().dbg_get_probe_stats(self.handle, ctypes.byref(s)), "dbg_get_probe_stats")
        return s.as_dict()


def build_batch(graphs: list[Graph], inputs: list[tuple], stream=None) -> list[int]:
    """``dbg_build_batch``: inputs[i] = (reads, offsets, k) for graphs[i].
    Returns the per-graph status codes."""
    m = len(graphs)
    keep = []
    arr = (Input * max(m, 1))()
    for i, (reads, offsets, k) in enumerate(inputs):
        reads, offsets = _host_inputs(reads, offsets)
        keep.append((reads, offsets))
        arr[i].reads = reads.ctypes.data if reads.size else None
        arr[i].offsets = offsets.ctypes.data if offsets.size else None
        arr[i].n_reads = max(0, offsets.shape[0] - 1)
        arr[i].k = int(k)
    hs = (ctypes.c_void_p * max(m, 1))(*[g.handle for g in graphs])
    st = (ctypes.c_int32 * max(m, 1))()
    lib().dbg_build_batch(hs, arr, m, st, _stream(stream))
    return [int(st[i]) for i in range(m)]


def build_batch_device(graphs: list[Graph], read_begin, ks, d_reads, d_offsets,
                       reads_len: int | None = None, stream=None) -> list[int]:
    """``dbg_build_batch_device`` over one device-resident concatenation."""
    m = len(graphs)
    rb = np.ascontiguousarray(read_begin, dtype=np.uint64)
    kk = np.ascontiguousarray(ks, dtype=np.uint32)
    assert rb.shape[0] == m + 1 and kk.shape[0] == m
    hs = (ctypes.c_void_p * max(m, 1))(*[g.handle for g in graphs])
    st = (ctypes.c_int32 * max(m, 1))()
    ln = int(d_reads.numel()) if reads_len is None else int(reads_len)
    lib().dbg_build_batch_device(hs, m, rb.ctypes.data, kk.ctypes.data, _ptr(d_reads), ln,
                                 _ptr(d_offsets), st, _stream(stream))
    return [int(st[i]) for i in range(m)]


def autotune(read_begin, ks, d_reads, d_offsets, expected_vertices=None, keep_flags: int = 0,
             repeats: int = 0, force: bool = False, reads_len: int | None = None,
             device: int = -1) -> Tuning:
    """``dbg_autotune`` over m instances laid out as in ``build_batch_device``
    (m = 1: a plain build).  Returns the chosen ``Tuning``; apply it with
    ``Graph(**t.graph_kwargs())`` (OR in the flags you keep)."""
    rb = np.ascontiguousarray(read_begin, dtype=np.uint64)
    kk = np.ascontiguousarray(ks, dtype=np.uint32)
    m = kk.shape[0]
    assert rb.shape[0] == m + 1
    ev = None if expected_vertices is None else np.ascontiguousarray(expected_vertices, dtype=np.uint64)
    t = Tuning()
    ln = int(d_reads.numel()) if reads_len is None else int(reads_len)
    rc = lib().dbg_autotune(int(device), m, rb.ctypes.data, kk.ctypes.data,
                            None if ev is None else ev.ctypes.data, _ptr(d_reads), ln, _ptr(d_offsets),
                            int(keep_flags), int(repeats), TUNE_FORCE if force else 0, ctypes.byref(t))
    _check(rc, "dbg_autotune")
    return t


def autotune_space(binned: bool) -> list[Tuning]:
    """``dbg_autotune_space``: every configuration the tuner may time for the
    binned or the direct build."""
    n = ctypes.c_uint32(0)
    _check(lib().dbg_autotune_space(1 if binned else 0, None, 0, ctypes.byref(n)), "dbg_autotune_space")
    arr = (Tuning * max(n.value, 1))()
    _check(lib().dbg_autotune_space(1 if binned else 0, arr, n.value, ctypes.byref(n)), "dbg_autotune_space")
    return [arr[i] for i in range(n.value)]


ROOF_LOAD64, ROOF_ADD32, ROOF_CAS64, ROOF_LOAD_ADD, ROOF_COPY = 0, 1, 2, 3, 4


def atomic_roofline(kind: int, footprint_bytes: int, n_ops: int, block_size: int = 256,
                    repeats: int = 5, device: int = -1) -> float:
    """Median kernel ms of n_ops random operations of `kind` over the footprint."""
    ms = ctypes.c_double(0)
    rc = lib().dbg_atomic_roofline(int(device), int(kind), int(footprint_bytes), int(n_ops),
                                   int(block_size), int(repeats), ctypes.byref(ms))
    _check(rc, "dbg_atomic_roofline")
    return float(ms.value)


class Server:
    """A build server (``dbg_server_create`` .. ``dbg_server_destroy``): FIFO
    admission against an HBM budget for tables, continuous batching of the
    admitted requests, tables resident until ``release``."""

    def __init__(self, hbm_budget: int = 0, max_batch: int = 0, max_batch_bytes: int = 0,
                 flags: int = 0, load_factor: float = 0.0, device: int = -1, slots: int = 0):
        cfg = ServerConfig()
        cfg.hbm_budget = int(hbm_budget)
        cfg.max_batch_bytes = int(max_batch_bytes)
        cfg.max_batch = int(max_batch)
        cfg.flags = int(flags)
        cfg.load_factor = float(load_factor)
        cfg.device = int(device)
        cfg.slots = int(slots)
        h = ctypes.c_void_p()
        _check(lib().dbg_server_create(ctypes.byref(cfg), ctypes.byref(h)), "dbg_server_create")
        self._h = h
        self._keep = {}

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("server is closed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().dbg_server_destroy(self._h)
            self._h = None
            self._keep = {}

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, reads, offsets, k: int, expected_vertices: int = 0) -> int:
        """Queue host-resident reads (copied); returns the request id."""
        reads, offsets = _host_inputs(reads, offsets)
        n = max(0, offsets.shape[0] - 1)
        rid = ctypes.c_uint64(0)
        rc = lib().dbg_server_submit(self.handle, reads.ctypes.data if reads.size else None,
                                     offsets.ctypes.data if offsets.size else None, n, int(k),
                                     int(expected_vertices), ctypes.byref(rid))
        _check(rc, "dbg_server_submit")
        return int(rid.value)

    def submit_device(self, d_reads, d_offsets, k: int, expected_vertices: int = 0,
                      n_reads: int | None = None, reads_len: int | None = None) -> int:
        """Queue device-resident reads; the tensors are kept alive until the
        request is released."""
        n = int(d_offsets.numel() - 1) if n_reads is None else int(n_reads)
        ln = int(d_reads.numel()) if reads_len is None else int(reads_len)
        rid = ctypes.c_uint64(0)
        rc = lib().dbg_server_submit_device(self.handle, _ptr(d_reads), ln, _ptr(d_offsets), n, int(k),
                                            int(expected_vertices), ctypes.byref(rid))
        _check(rc, "dbg_server_submit_device")
        self._keep[int(rid.value)] = (d_reads, d_offsets)
        return int(rid.value)

    def poll(self, rid: int) -> int | None:
        """None while pending, else the request's build status."""
        st = ctypes.c_int32(0)
        rc = lib().dbg_server_poll(self.handle, int(rid), ctypes.byref(st))
        if rc == PENDING:
            return None
        _check(rc, "dbg_server_poll")
        return int(st.value)

    def wait(self, rid: int, timeout: float = -1.0) -> int | None:
        """The request's build status; None if the timeout passed first."""
        st = ctypes.c_int32(0)
        rc = lib().dbg_server_wait(self.handle, int(rid), float(timeout), ctypes.byref(st))
        if rc == PENDING:
            return None
        _check(rc, "dbg_server_wait")
        return int(st.value)

    def graph(self, rid: int) -> Graph:
        """The finished request's graph (owned by the server until release)."""
        h = ctypes.c_void_p()
        _check(lib().dbg_server_graph(self.handle, int(rid), ctypes.byref(h)), "dbg_server_graph")
        return Graph(_borrowed=h.value)

    def times(self, rid: int) -> tuple[float, float, float]:
        """(submitted, started, finished) in seconds on the server's clock."""
        a, b, c = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        rc = lib().dbg_server_times(self.handle, int(rid), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        if rc not in (OK, PENDING):
            _check(rc, "dbg_server_times")
        return float(a.value), float(b.value), float(c.value)

    def release(self, rid: int) -> None:
        _check(lib().dbg_server_release(self.handle, int(rid)), "dbg_server_release")
        self._keep.pop(int(rid), None)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().dbg_server_get_stats(self.handle, ctypes.byref(s)), "dbg_server_get_stats")
        return s.as_dict()
