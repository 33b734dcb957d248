"""Parity of the HIP build (through the C ABI) with the CPU oracle.

Integer work, so the bar is bit-exact: the sorted (key, counts[4]) records of
the device graph must equal the oracle's.  Table layout and extract order are
free; the records are sorted before comparison.
"""

import numpy as np
import pytest

import oracle
import readsim
import paper_2401_02756_amd as dbg
from oracle import invariants

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def say(msg):
    print("[case] " + msg, flush=True)


def assert_same(got, want, what=""):
    gk, gc = got
    wk, wc = want
    assert gk.shape == wk.shape, "%s: %d vertices, oracle has %d" % (what, gk.shape[0], wk.shape[0])
    bad_k = int(np.count_nonzero(gk != wk))
    assert bad_k == 0, "%s: %d keys differ" % (what, bad_k)
    bad_c = int(np.count_nonzero(np.any(gc != wc, axis=1)))
    assert bad_c == 0, "%s: %d vertices have different counts" % (what, bad_c)


def gpu_build(rs, **kw):
    with dbg.Graph(**kw) as g:
        g.build(rs.reads, rs.offsets, rs.k)
        return g.extract_sorted()


def gpu_build_device(rs, **kw):
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    with dbg.Graph(**kw) as g:
        g.build_device(d_reads, d_off, rs.k)
        g.sync()
        return g.extract_sorted()


def oracle_of(rs):
    return oracle.build_graph(rs.reads, rs.offsets, rs.k)


# ---------------------------------------------------------------- the paper's example

def test_worked_example(worked_example):
    read, k, verts = worked_example
    say("worked example ACGACGACGC k=4")
    rs = readsim.reads_from_strings([read], k)
    keys, counts = gpu_build(rs)
    got = {oracle.decode_key(x, k): (int(x), c.tolist()) for x, c in zip(keys, counts)}
    assert got == verts


# ---------------------------------------------------------------- configuration 1

MODES = [0, dbg.F_BINNED]
MODE_IDS = ["direct", "binned"]

SHAPES = [
    dict(),
    dict(flags=dbg.F_BINNED),
    dict(flags=dbg.F_BINNED | dbg.F_ENTRY32),
    dict(block_size=64, windows_per_thread=1),
    dict(block_size=1024, windows_per_thread=2),
    dict(block_size=256, windows_per_thread=16),
    dict(flags=dbg.F_MERGE),
    dict(flags=dbg.F_MERGE, block_size=1024, windows_per_thread=1),
    dict(flags=dbg.F_ENTRY32),
    dict(flags=dbg.F_ENTRY32 | dbg.F_MERGE, block_size=512),
]


@pytest.fixture(scope="module")
def config1():
    rs = readsim.make_config(1)
    return rs, oracle_of(rs)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "-".join("%s%s" % kv for kv in s.items()) or "default")
def test_config1_launch_shapes(config1, shape):
    rs, want = config1
    say("config1 host build %r" % shape)
    assert_same(gpu_build(rs, **shape), want, "config1 %r" % shape)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_config1_device_build(config1, mode):
    rs, want = config1
    say("config1 device build mode %d" % mode)
    assert_same(gpu_build_device(rs, flags=mode), want, "config1 device")


@pytest.mark.parametrize("lf", [0.3, 0.7, 0.85, 0.95])
def test_config1_load_factors(config1, lf):
    rs, want = config1
    say("config1 load factor %.2f" % lf)
    V = want[0].shape[0]
    assert_same(gpu_build(rs, capacity=int(V / lf) + 1), want, "lf %.2f" % lf)
    if lf <= dbg.BINNED_MAX_LOAD:  # a binned table fails when one 2048-slot segment overflows
        assert_same(gpu_build(rs, capacity=int(V / lf) + 1, flags=dbg.F_BINNED), want, "binned lf %.2f" % lf)
        assert_same(gpu_build(rs, expected_vertices=V, load_factor=lf, flags=dbg.F_BINNED), want,
                    "binned, load factor %.2f" % lf)


def test_config1_stats_and_timing(config1):
    rs, want = config1
    with dbg.Graph(flags=dbg.F_TIMING, expected_vertices=20000) as g:
        g.build(rs.reads, rs.offsets, rs.k)
        st = g.stats()
    assert st["vertices"] == want[0].shape[0]
    assert st["inserts"] == invariants.expected_total(rs.offsets, rs.k) == int(want[1].sum())
    assert st["k"] == rs.k and st["builds"] == 1 and st["status"] == 0
    assert st["last_build_ms"] > 0 and st["last_total_ms"] >= st["last_build_ms"]
    assert st["entry_bytes"] == 24 and st["capacity"] == 40000


def test_repeated_runs_identical(config1):
    rs, want = config1
    say("config1 determinism x3, tight table")
    V = want[0].shape[0]
    for _ in range(3):
        assert_same(gpu_build(rs, capacity=V + V // 16), want, "repeat")
        assert_same(gpu_build(rs, capacity=int(V / 0.7), flags=dbg.F_BINNED), want, "repeat binned")


def test_binned_reset_does_not_leak_old_contents(config1):
    rs, want = config1
    say("binned: lazy reset between two different builds")
    other = readsim.make_config(2, scale=0.002)
    other.k = rs.k
    with dbg.Graph(flags=dbg.F_BINNED, expected_vertices=60000) as g:
        g.build(other.reads, other.offsets, rs.k)
        g.reset()
        assert g.vertex_count() == 0
        g.build(rs.reads, rs.offsets, rs.k)
        got = g.extract_sorted()
    assert_same(got, want, "after reset")


def test_binned_k32_falls_back_to_direct():
    say("binned graph with k=32")
    rng = np.random.default_rng(32)
    reads = ["".join(rng.choice(list("ACGT"), size=120)) for _ in range(500)]
    rs = readsim.reads_from_strings(reads, 32)
    want = oracle_of(rs)
    with dbg.Graph(flags=dbg.F_BINNED) as g:
        g.build(rs.reads, rs.offsets, 32)
        got = g.extract_sorted()
    assert_same(got, want, "k=32 binned graph")


# ---------------------------------------------------------------- edge cases

def test_empty_and_short_inputs():
    say("empty / short reads")
    with dbg.Graph() as g:
        g.build(np.zeros(0, np.uint8), np.zeros(1, np.uint64), 5)
        assert g.vertex_count() == 0
        rs = readsim.reads_from_strings(["", "ACG", "ACGT"], 5)  # all shorter than k
        g.build(rs.reads, rs.offsets, 5)
        assert g.vertex_count() == 0
        rs = readsim.reads_from_strings(["ACGTA"], 5)  # exactly k: two vertices, one edge
        g.build(rs.reads, rs.offsets, 5)
        keys, counts = g.extract_sorted()
    assert sorted(oracle.decode_key(x, 5) for x in keys) == ["ACGT", "CGTA"]
    assert int(counts.sum()) == 1


@pytest.mark.parametrize("k", [2, 3, 5, 17, 21, 31, 32])
def test_ragged_reads_all_k(k):
    say("ragged reads k=%d" % k)
    rng = np.random.default_rng(k)
    lens = rng.integers(0, 300, size=3000)
    lens[::97] = k - 1
    lens[::89] = k
    reads = ["".join(rng.choice(list("ACGTacgt"), size=int(L))) for L in lens]
    rs = readsim.reads_from_strings(reads, k)
    want = oracle_of(rs)
    assert_same(gpu_build(rs), want, "ragged k=%d" % k)
    assert_same(gpu_build(rs, flags=dbg.F_MERGE, block_size=128, windows_per_thread=3), want,
                "ragged merged k=%d" % k)
    assert_same(gpu_build(rs, flags=dbg.F_BINNED), want, "ragged binned k=%d" % k)


def test_offsets_not_starting_at_zero():
    say("offsets start past the first byte")
    rs = readsim.make_config(1)
    pad = 77
    reads = np.concatenate([np.full(pad, ord("N"), np.uint8), rs.reads])
    offsets = rs.offsets + np.uint64(pad)
    want = oracle_of(rs)
    with dbg.Graph() as g:
        g.build(reads, offsets, rs.k)
        got = g.extract_sorted()
    assert_same(got, want, "host offsets with a base")
    with dbg.Graph(flags=dbg.F_BINNED) as g:
        g.build(reads, offsets, rs.k)
        got = g.extract_sorted()
    assert_same(got, want, "binned host offsets with a base")
    # device slice of a larger concatenation
    d_reads = torch.from_numpy(reads[pad:]).cuda()
    d_off = torch.from_numpy(offsets.astype(np.int64)).cuda()
    with dbg.Graph() as g:
        g.build_device(d_reads, d_off, rs.k)
        g.sync()
        got = g.extract_sorted()
    assert_same(got, want, "device offsets with a base")


def test_hot_key_poly_a_and_tandem_repeats():
    say("hot keys: poly-A and tandem repeats")
    reads = ["A" * 150] * 5000 + ["AC" * 75] * 3000 + ["ACGTT" * 30] * 3000 + ["GATTACA" * 21] * 1000
    rs = readsim.reads_from_strings(reads, 31)
    want = oracle_of(rs)
    assert_same(gpu_build(rs), want, "hot keys")
    assert_same(gpu_build(rs, flags=dbg.F_MERGE), want, "hot keys merged")
    assert_same(gpu_build(rs, flags=dbg.F_MERGE, block_size=64, windows_per_thread=1), want,
                "hot keys merged wave64")
    assert_same(gpu_build(rs, flags=dbg.F_BINNED), want, "hot keys binned")
    assert int(want[1].max()) == 5000 * 120


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_incremental_builds_accumulate(config1, mode):
    rs, want = config1
    say("incremental: two halves, mode %d" % mode)
    h = rs.n_reads // 2
    a = readsim.reads_from_strings([rs.read(i) for i in range(h)], rs.k)
    b = readsim.reads_from_strings([rs.read(i) for i in range(h, rs.n_reads)], rs.k)
    with dbg.Graph(expected_vertices=20000, flags=mode) as g:
        g.build(a.reads, a.offsets, rs.k)
        g.build(b.reads, b.offsets, rs.k)
        got = g.extract_sorted()
        assert g.stats()["builds"] == 2
    assert_same(got, want, "two halves")


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_full_table_is_reported_and_poisons(mode):
    say("undersized table -> FULL, mode %d" % mode)
    rs = readsim.make_config(1)
    with dbg.Graph(capacity=1000, flags=mode) as g:
        with pytest.raises(dbg.DbgError) as e:
            g.build(rs.reads, rs.offsets, rs.k)
        assert e.value.code == dbg.E_FULL
        assert g.stats()["status"] == dbg.E_FULL
        with pytest.raises(dbg.DbgError) as e:
            g.build(rs.reads, rs.offsets, rs.k)
        assert e.value.code == dbg.E_STATE
        keys, counts = g.extract()  # partial graph is still readable
        assert keys.shape[0] <= g.stats()["capacity"]
        g.reset()
        g.build(readsim.reads_from_strings(["ACGTACGT"], 5).reads,
                readsim.reads_from_strings(["ACGTACGT"], 5).offsets, 5)
        assert g.vertex_count() == 4


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_rejected_inputs_modify_nothing(config1, mode):
    rs, want = config1
    say("bad base / bad k / bad offsets leave the graph unchanged, mode %d" % mode)
    with dbg.Graph(expected_vertices=20000, flags=mode) as g:
        g.build(rs.reads, rs.offsets, rs.k)
        bad = readsim.reads_from_strings(["ACGTACGTACGTACGTACGTACGTACGTNACGT"] * 10, rs.k)
        with pytest.raises(dbg.DbgError) as e:
            g.build(bad.reads, bad.offsets, rs.k)
        assert e.value.code == dbg.E_BASE
        with pytest.raises(dbg.DbgError) as e:
            g.build(rs.reads, rs.offsets, rs.k + 1)
        assert e.value.code == dbg.E_K
        with pytest.raises(dbg.DbgError) as e:
            g.build(rs.reads, rs.offsets[::-1].copy(), rs.k)
        assert e.value.code == dbg.E_INVAL
        # device-side offset check
        d_reads = torch.from_numpy(rs.reads).cuda()
        off = rs.offsets.astype(np.int64).copy()
        off[5], off[6] = off[6], off[5]
        d_off = torch.from_numpy(off).cuda()
        g.build_device(d_reads, d_off, rs.k)
        with pytest.raises(dbg.DbgError) as e:
            g.sync()
        assert e.value.code == dbg.E_INVAL
        # device-side byte check
        bad_reads = rs.reads.copy()
        bad_reads[12345] = ord("x")
        g.build_device(torch.from_numpy(bad_reads).cuda(),
                       torch.from_numpy(rs.offsets.astype(np.int64)).cuda(), rs.k)
        with pytest.raises(dbg.DbgError) as e:
            g.sync()
        assert e.value.code == dbg.E_BASE
        got = g.extract_sorted()
        assert g.stats()["builds"] == 1
    assert_same(got, want, "after rejected inputs")


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_extract_space_and_device_extract(config1, mode):
    rs, want = config1
    say("extract: too small buffer, device buffers, mode %d" % mode)
    import ctypes
    with dbg.Graph(flags=mode) as g:
        g.build(rs.reads, rs.offsets, rs.k)
        V = g.vertex_count()
        keys = np.empty(V - 1, np.uint64)
        counts = np.empty((V - 1, 4), np.uint32)
        n = ctypes.c_uint64()
        rc = dbg.lib().dbg_extract(g.handle, keys.ctypes.data, counts.ctypes.data, V - 1,
                                   ctypes.byref(n))
        assert rc == dbg.E_SPACE and n.value == V
        dk = torch.empty(V, dtype=torch.int64, device="cuda")
        dc = torch.empty((V, 4), dtype=torch.int32, device="cuda")
        assert g.extract_device(dk, dc) == V
        torch.cuda.synchronize()
        k2 = dk.cpu().numpy().view(np.uint64)
        c2 = dc.cpu().numpy().view(np.uint32)
    order = np.argsort(k2)
    assert_same((k2[order], c2[order]), want, "device extract")


# ---------------------------------------------------------------- configuration 2

def test_config2_scaled():
    rs = readsim.make_config(2, scale=0.05)
    say("config2 at 5%% scale (%d reads)" % rs.n_reads)
    want = oracle_of(rs)
    assert_same(gpu_build(rs, expected_vertices=rs.meta["expected_vertices"]), want, "config2 5%")
    assert_same(gpu_build(rs, flags=dbg.F_MERGE), want, "config2 5% merged")
    assert_same(gpu_build(rs, flags=dbg.F_BINNED, expected_vertices=rs.meta["expected_vertices"]), want,
                "config2 5% binned")


# ---------------------------------------------------------------- batched

@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_batch_matches_per_instance_oracle(mode):
    say("batched build of 12 small instances + failures, mode %d" % mode)
    sets = []
    for j in range(40):
        p = readsim.instance_params(4, j)
        if p["genome_len"] < 60_000:
            sets.append(readsim.make_instance(4, j))
        if len(sets) == 12:
            break
    assert len(sets) >= 6
    bad = readsim.reads_from_strings(["ACGTNNACGT" * 5], 21)
    graphs = [dbg.Graph(flags=mode) for _ in range(len(sets) + 1)]
    inputs = [(rs.reads, rs.offsets, rs.k) for rs in sets] + [(bad.reads, bad.offsets, 21)]
    try:
        st = dbg.build_batch(graphs, inputs)
        assert st[:-1] == [0] * len(sets), st
        assert st[-1] == dbg.E_BASE
        assert graphs[-1].vertex_count() == 0
        for rs, g in zip(sets, graphs):
            assert_same(g.extract_sorted(), oracle_of(rs), "batch instance")
        # a second batch adds to the same graphs (counts double)
        st = dbg.build_batch(graphs[:-1], inputs[:-1])
        assert st == [0] * len(sets)
        for rs, g in zip(sets, graphs):
            k2, c2 = g.extract_sorted()
            wk, wc = oracle_of(rs)
            assert np.array_equal(k2, wk) and np.array_equal(c2, 2 * wc)
    finally:
        for g in graphs:
            g.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_batch_device_matches_plain_device(mode):
    say("batched device build vs plain device builds on slices, mode %d" % mode)
    sets = [readsim.make_instance(4, j) for j in range(6)]
    sets = [s for s in sets if s.total_bases < 40_000_000]
    reads = np.concatenate([s.reads for s in sets])
    lens = np.concatenate([s.lengths() for s in sets])
    offs = np.zeros(lens.shape[0] + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    rb = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([s.n_reads for s in sets], out=rb[1:])
    ks = [s.k for s in sets]
    d_reads = torch.from_numpy(reads).cuda()
    d_off = torch.from_numpy(offs).cuda()
    graphs = [dbg.Graph(flags=mode) for _ in sets]
    try:
        st = dbg.build_batch_device(graphs, rb, ks, d_reads, d_off)
        assert st == [0] * len(sets)
        for i, (s, g) in enumerate(zip(sets, graphs)):
            got = g.extract_sorted()
            b0, b1 = int(offs[rb[i]]), int(offs[rb[i + 1]])
            with dbg.Graph(flags=mode) as p:
                p.build_device(d_reads[b0:b1], d_off[int(rb[i]):int(rb[i + 1]) + 1], s.k)
                p.sync()
                plain = p.extract_sorted()
            assert_same(got, plain, "batched vs plain %d" % i)
            assert_same(got, oracle_of(s), "batched vs oracle %d" % i)
    finally:
        for g in graphs:
            g.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_batch_unsized_graphs_sized_from_own_input(mode):
    """A graph created without a size is sized, in a batch as in dbg_build,
    from its own input (ceil(bound / load factor) slots, bound = its windows
    from host input, its bytes from device input), not from the whole
    concatenation."""
    say("batched build of unsized graphs: each table sized from its own input, mode %d" % mode)
    sets = [readsim.make_instance(4, j) for j in range(8)]
    sets = [s for s in sets if s.total_bases < 40_000_000][:5]
    lf = 0.5

    def windows(s):
        L = s.lengths()
        return int(np.where(L >= s.k, L - s.k + 2, 0).sum())

    def check(graphs, bounds, what):
        for i, (s, g, b) in enumerate(zip(sets, graphs, bounds)):
            own = max(64, 2 * b)  # ceil(b / 0.5)
            cap = g.stats()["capacity"]
            if mode == dbg.F_BINNED:  # whole segments, a few more than asked for
                assert own <= cap <= own + 64 * 2048 + own // 8, (what, i, cap, own)
            else:
                assert cap == own, (what, i, cap, own)
            assert_same(g.extract_sorted(), oracle_of(s), "%s instance %d" % (what, i))

    graphs = [dbg.Graph(load_factor=lf, flags=mode) for _ in sets]
    try:
        assert dbg.build_batch(graphs, [(s.reads, s.offsets, s.k) for s in sets]) == [0] * len(sets)
        check(graphs, [windows(s) for s in sets], "host input")
    finally:
        for g in graphs:
            g.close()
    reads = np.concatenate([s.reads for s in sets])
    lens = np.concatenate([s.lengths() for s in sets])
    offs = np.zeros(lens.shape[0] + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    rb = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([s.n_reads for s in sets], out=rb[1:])
    graphs = [dbg.Graph(load_factor=lf, flags=mode) for _ in sets]
    try:
        st = dbg.build_batch_device(graphs, rb, [s.k for s in sets], torch.from_numpy(reads).cuda(),
                                    torch.from_numpy(offs).cuda())
        assert st == [0] * len(sets)
        check(graphs, [int(s.total_bases) for s in sets], "device input")
    finally:
        for g in graphs:
            g.close()


# ---------------------------------------------------------------- graph capture and replay

@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_graph_replays_match_eager(mode):
    say("graph capture + replays vs eager, mode %d" % mode)
    a = readsim.make_config(1)
    b = readsim.simulate(10_000, 100, 10.0, 0.005, 21, 77)  # same size class, other data
    want_a, want_b = oracle_of(a), oracle_of(b)
    eager = gpu_build(a, flags=mode)
    assert_same(eager, want_a, "eager")
    da = (torch.from_numpy(a.reads).cuda(), torch.from_numpy(a.offsets.astype(np.int64)).cuda())
    db = (torch.from_numpy(b.reads).cuda(), torch.from_numpy(b.offsets.astype(np.int64)).cuda())
    with dbg.Graph(flags=mode | dbg.F_GRAPH, expected_vertices=20000) as g:
        for rep in range(4):
            for (dr, do), rs, want in ((da, a, want_a), (db, b, want_b)):
                g.reset()
                g.build_device(dr, do, rs.k)
                g.sync()
                assert_same(g.extract_sorted(), want, "replay %d" % rep)
                # eager work and a sync between replays
                x = torch.arange(1 << 20, device="cuda", dtype=torch.int64).sum()
                torch.cuda.synchronize()
                assert int(x) == (1 << 20) * ((1 << 20) - 1) // 2
        st = g.stats()
    assert st["graph_captures"] >= 1 and st["graph_replays"] >= 6, st


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_graph_batch_replays(mode):
    say("batched build through graphs, mode %d" % mode)
    sets = [readsim.make_instance(4, j) for j in range(3)]
    sets = [s for s in sets if s.total_bases < 30_000_000]
    wants = [oracle_of(s) for s in sets]
    for rep in range(3):
        graphs = [dbg.Graph(flags=mode | dbg.F_GRAPH) for _ in sets]
        try:
            st = dbg.build_batch(graphs, [(s.reads, s.offsets, s.k) for s in sets])
            assert st == [0] * len(sets)
            for g, want in zip(graphs, wants):
                assert_same(g.extract_sorted(), want, "batch replay %d" % rep)
        finally:
            for g in graphs:
                g.close()


# ---------------------------------------------------------------- measurement kernel

def test_roofline_kernel_runs():
    for kind in range(4):
        ms = dbg.atomic_roofline(kind, 1 << 24, 1 << 20, 256, 2)
        assert ms > 0
