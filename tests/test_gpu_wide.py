"""Long k (33 <= k <= 64) on the device against the oracle's 128-bit build.

Keys come back as two words (K >> 64, K mod 2^64); the comparison is exact on
the sorted (high, low, counts) records.
"""

import numpy as np
import pytest

import oracle
import readsim
import paper_2401_02756_amd as dbg

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


def want(rs, k):
    hi, lo, counts = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    return np.stack([hi, lo], axis=1), counts


def check(got, exp):
    gk, gc = got
    ek, ec = exp
    assert gk.shape == ek.shape, (gk.shape, ek.shape)
    assert np.array_equal(gk, ek)
    assert np.array_equal(gc, ec)


MODES = [0, dbg.F_BINNED]
MODE_IDS = ["direct", "binned"]


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("k", [33, 40, 51, 63, 64])
def test_random_reads(k, mode):
    rs = readsim.simulate(200_000, 150, 12.0, 0.01, k, 900 + k)
    say("long k=%d random reads, mode %d" % (k, mode))
    with dbg.Graph(flags=mode) as g:
        g.build(rs.reads, rs.offsets, k)
        check(g.extract_sorted(), want(rs, k))
        # binned graphs stay binned up to k = 63
        assert g.stats()["entry_bytes"] == 32 and g.stats()["binned"] == (1 if mode and k <= 63 else 0)


def test_ragged_and_edge_reads():
    rng = np.random.default_rng(5)
    alphabet = np.array(list(b"ACGTacgt"), dtype=np.uint8)
    reads = []
    for _ in range(3000):
        n = int(rng.integers(0, 200))
        reads.append(alphabet[rng.integers(0, 8, n)].tobytes())
    reads += [b"", b"A" * 50, b"C" * 51, b"G" * 52, b"ACGT" * 60]
    for k in (33, 51, 63, 64):
        rs = readsim.reads_from_strings(reads, k)
        exp = want(rs, k)
        for mode in MODES:
            say("long k=%d ragged, mode %d" % (k, mode))
            with dbg.Graph(flags=mode) as g:
                g.build(rs.reads, rs.offsets, k)
                check(g.extract_sorted(), exp)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_one_key_everywhere(mode):
    # every window of every read is the same vertex: all lanes race for one slot
    k = 51
    rs = readsim.reads_from_strings([b"A" * 150] * 4000 + [b"AC" * 75] * 4000, k)
    say("long k contended claims, mode %d" % mode)
    with dbg.Graph(flags=mode) as g:
        g.build(rs.reads, rs.offsets, k)
        check(g.extract_sorted(), want(rs, k))


def test_shared_prefixes_on_a_crowded_table():
    # keys that share their first 40 bases and differ only at the end, in a
    # table filled to about 80 %: long probe chains over similar keys
    rng = np.random.default_rng(17)
    k = 45
    stem = "".join("ACGT"[x] for x in rng.integers(0, 4, 40))
    reads = [stem + "".join("ACGT"[x] for x in rng.integers(0, 4, 30)) for _ in range(3000)]
    rs = readsim.reads_from_strings(reads, k)
    exp = want(rs, k)
    for mode in MODES:
        say("long k shared prefixes, mode %d" % mode)
        with dbg.Graph(flags=mode, expected_vertices=90_000, load_factor=0.85) as g:
            g.build(rs.reads, rs.offsets, k)
            check(g.extract_sorted(), exp)


def test_device_input_binned_flag_and_accumulation():
    k = 51
    rs = readsim.simulate(300_000, 150, 10.0, 0.01, k, 77)
    say("long k device input, binned flag, two builds")
    exp = want(rs, k)
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    half = rs.n_reads // 2
    ev = readsim.expected_vertices(300_000, 150, rs.n_reads, 0.01, k)
    with dbg.Graph(flags=dbg.F_BINNED | dbg.F_GRAPH, expected_vertices=ev) as g:
        # two halves from one device concatenation; counts add up
        g.build_device(d_reads, d_off[:half + 1], k, reads_len=int(rs.offsets[half]))
        g.build_device(d_reads[int(rs.offsets[half]):], d_off[half:], k)
        g.sync()
        check(g.extract_sorted(), exp)
        V = g.vertex_count()
        d_keys = torch.empty(2 * V, dtype=torch.int64, device="cuda")
        d_cnt = torch.empty(4 * V, dtype=torch.int32, device="cuda")
        assert g.extract_device(d_keys, d_cnt) == V
        keys = d_keys.cpu().numpy().view(np.uint64).reshape(V, 2)
        cnt = d_cnt.cpu().numpy().view(np.uint32).reshape(V, 4)
        order = np.lexsort((keys[:, 1], keys[:, 0]))
        check((keys[order], cnt[order]), exp)
        # too small an output buffer
        with pytest.raises(dbg.DbgError) as e:
            g.extract_device(d_keys[:-2], d_cnt)
        assert e.value.code == dbg.E_SPACE


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_reset_to_short_k_and_back(mode):
    rs = readsim.simulate(100_000, 150, 8.0, 0.01, 21, 31)
    say("long k then k=21 on one handle, mode %d" % mode)
    with dbg.Graph(flags=mode, expected_vertices=readsim.expected_vertices(100_000, 150, rs.n_reads, 0.01, 45)) as g:
        g.build(rs.reads, rs.offsets, 45)
        check(g.extract_sorted(), want(rs, 45))
        with pytest.raises(dbg.DbgError) as e:
            g.build(rs.reads, rs.offsets, 21)  # k differs from the graph's
        assert e.value.code == dbg.E_K
        g.reset()
        g.build(rs.reads, rs.offsets, 21)
        keys, counts = g.extract_sorted()
        ek, ec = oracle.build_graph(rs.reads, rs.offsets, 21)
        assert np.array_equal(keys, ek) and np.array_equal(counts, ec)
        g.reset()
        g.build(rs.reads, rs.offsets, 64)
        check(g.extract_sorted(), want(rs, 64))


def test_errors_and_limits():
    rs = readsim.simulate(20_000, 150, 5.0, 0.01, 51, 3)
    with dbg.Graph() as g:
        with pytest.raises(dbg.DbgError) as e:
            g.build(rs.reads, rs.offsets, 65)
        assert e.value.code == dbg.E_K
        g.build(rs.reads, rs.offsets, 51)
        with pytest.raises(dbg.DbgError) as e:
            g.contig_sizes()
        assert e.value.code == dbg.E_K
        kk, cc = g.extract_normalized(20_000)
        ek, ec = want(rs, 51)
        order = np.lexsort((kk[:, 1], kk[:, 0]))
        assert np.array_equal(kk[order], ek)
        assert np.array_equal(cc[order], oracle.normalize(ec, 20_000, int(ec.sum()))[0])
    # batches keep k <= 32
    with dbg.Graph() as g:
        st = dbg.build_batch([g], [(rs.reads, rs.offsets, 40)])
        assert st == [dbg.E_K]
    bad = readsim.reads_from_strings([b"ACGT" * 20 + b"N" + b"ACGT" * 20], 51)
    for mode in MODES:
        # a table too small for the vertices (one segment when binned): full, poisoned
        with dbg.Graph(capacity=1000, flags=mode) as g:
            with pytest.raises(dbg.DbgError) as e:
                g.build(rs.reads, rs.offsets, 51)
            assert e.value.code == dbg.E_FULL
            with pytest.raises(dbg.DbgError) as e:
                g.build(rs.reads, rs.offsets, 51)
            assert e.value.code == dbg.E_STATE
        with dbg.Graph(flags=mode) as g:
            with pytest.raises(dbg.DbgError) as e:
                g.build(bad.reads, bad.offsets, 51)
            assert e.value.code == dbg.E_BASE
            assert g.vertex_count() == 0
            g.build(rs.reads, rs.offsets, 51)  # a rejected input leaves the graph usable
            check(g.extract_sorted(), want(rs, 51))


def test_autotune_long_k():
    k = 51
    rs = readsim.simulate(200_000, 150, 10.0, 0.01, k, 12)
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    say("long k autotune")
    t = dbg.autotune([0, rs.n_reads], [k], d_reads, d_off, repeats=1)
    assert t.flags & dbg.F_MERGE == 0  # the long-k direct build does not merge
    with dbg.Graph(**t.graph_kwargs()) as g:
        g.build(rs.reads, rs.offsets, k)
        check(g.extract_sorted(), want(rs, k))


@pytest.mark.timeout(900)
def test_bacterial_k51_exact():
    rs = readsim.make_config(2)
    k = 51
    say("long k=51 bacterial scale")
    exp = want(rs, k)
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    for mode in MODES:
        say("long k=51 bacterial scale, mode %d" % mode)
        with dbg.Graph(expected_vertices=readsim.expected_vertices(5_000_000, 150, rs.n_reads, 0.01, k),
                       load_factor=0.5, flags=dbg.F_GRAPH | mode) as g:
            g.build_device(d_reads, d_off, k)
            g.sync()
            check(g.extract_sorted(), exp)
