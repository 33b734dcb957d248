"""Stress of the find-or-claim paths and the probe statistics (DBG_F_STATS).

With DBG_F_TEST_HASH every key's home slot is the low 3 bits of its key (of
its image inside a binned segment), so every key of a table (of a segment)
walks one probe chain and every claim races with the others at the chain's
end: the retry path of the compare-and-swap (Algorithms 1 and 3 of the paper)
runs on nearly every claim.  The graphs must still equal the oracle's.  The
probe statistics must satisfy what any build satisfies: every lookup falls
in one histogram bin, one lookup per window (no merging), and, into an empty
table, one won compare-and-swap per vertex.
"""

import numpy as np
import pytest

import oracle
import readsim
import paper_2401_02756_amd as dbg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = [0, dbg.F_BINNED]
MODE_IDS = ["direct", "binned"]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def say(msg):
    print("[case] " + msg, flush=True)


def windows_of(rs, k):
    L = rs.lengths()
    return int(np.where(L >= k, L - k + 2, 0).sum())


def check_stats(ps, windows, vertices, what, fresh=True):
    assert sum(ps["probe_hist"]) == ps["lookups"], (what, ps)
    assert ps["lookups"] == windows, (what, ps, windows)
    assert ps["probes"] >= ps["lookups"], (what, ps)
    assert ps["cas_attempts"] >= ps["cas_lost"], (what, ps)
    if fresh:
        assert ps["cas_attempts"] - ps["cas_lost"] == vertices, (what, ps, vertices)


def hot_keys():
    reads = ["A" * 150] * 500 + ["AC" * 75] * 300 + ["ACGTT" * 30] * 300 + ["GATTACA" * 21] * 100
    return readsim.reads_from_strings(reads, 31)


def same(got, want, what):
    assert got[0].shape == want[0].shape, "%s: %d vertices, oracle has %d" % (what, got[0].shape[0],
                                                                            want[0].shape[0])
    assert np.array_equal(got[0], want[0]), what + ": keys differ"
    assert np.array_equal(got[1], want[1]), what + ": counts differ"


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("which", ["config1", "hot_keys"])
def test_one_probe_chain_equals_oracle(mode, which):
    rs = readsim.make_config(1) if which == "config1" else hot_keys()
    want = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    V = want[0].shape[0]
    say("test hash, %s, mode %d: %d vertices on one probe chain per %s" %
        (which, mode, V, "segment" if mode else "table"))
    with dbg.Graph(expected_vertices=V, load_factor=0.5, flags=mode | dbg.F_TEST_HASH | dbg.F_STATS) as g:
        g.build(rs.reads, rs.offsets, rs.k)
        same(g.extract_sorted(), want, "test hash, " + which)
        ps = g.probe_stats()
    check_stats(ps, windows_of(rs, rs.k), V, which)
    if which == "config1":  # thousands of vertices: the chain is long and claims race for its end
        assert ps["probes"] > 20 * ps["lookups"], ps
        assert ps["probe_hist"][7] > 0, ps
    say("  %s" % ps)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_one_probe_chain_long_k_and_batches(mode):
    # long k: the two-word claim (compare-and-swap of the first word, then the second) under the same races
    rng = np.random.default_rng(5)
    k = 45
    reads = ["".join("ACGT"[x] for x in rng.integers(0, 4, 90)) for _ in range(400)]
    rs = readsim.reads_from_strings(reads, k)
    hi, lo, c = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    say("test hash, long k = %d, mode %d: %d vertices" % (k, mode, hi.shape[0]))
    with dbg.Graph(expected_vertices=hi.shape[0], flags=mode | dbg.F_TEST_HASH | dbg.F_STATS) as g:
        g.build(rs.reads, rs.offsets, k)
        keys, counts = g.extract_sorted()
        ps = g.probe_stats()
    assert np.array_equal(keys[:, 0], hi) and np.array_equal(keys[:, 1], lo) and np.array_equal(counts, c)
    check_stats(ps, windows_of(rs, k), hi.shape[0], "long k")
    # a batch of test-hash graphs equals the oracle per graph; a graph of the
    # other setting in the same launch is refused (small sets: one probe chain
    # of a direct table stops at 65,536 slots, the build's probe limit)
    sets = [readsim.simulate(4000, 100, 10.0, 0.005, k2, seed=900 + k2) for k2 in (21, 31)]
    gs = [dbg.Graph(flags=mode | dbg.F_TEST_HASH) for _ in sets]
    other = dbg.Graph(flags=mode)
    try:
        st = dbg.build_batch(gs + [other], [(x.reads, x.offsets, x.k) for x in sets] +
                             [(sets[0].reads, sets[0].offsets, sets[0].k)])
        assert st[:2] == [0, 0] and st[2] == dbg.E_INVAL, st
        assert other.vertex_count() == 0
        for x, g in zip(sets, gs):
            same(g.extract_sorted(), oracle.build_graph(x.reads, x.offsets, x.k), "test-hash batch")
    finally:
        for g in gs + [other]:
            g.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_probe_stats_normal_hash(mode):
    rs = readsim.make_config(2)
    n = 100_000  # a tenth of the bacterial-scale reads
    end = int(rs.offsets[n])
    reads, offs = rs.reads[:end], rs.offsets[:n + 1]
    sub = readsim.ReadSet(reads=reads, offsets=offs, k=rs.k)
    want = oracle.build_graph_parallel(reads, offs, rs.k, threads=16)
    V = want[0].shape[0]
    say("probe statistics, scaled bacterial reads, mode %d" % mode)
    with dbg.Graph(expected_vertices=V, load_factor=0.5, flags=mode | dbg.F_STATS) as g:
        g.build(reads, offs, rs.k)
        same(g.extract_sorted(), want, "statistics build")
        ps = g.probe_stats()
        check_stats(ps, windows_of(sub, rs.k), V, "one build")
        # at load factor 0.5 linear probing stays short
        assert ps["probes"] < 2.0 * ps["lookups"], ps
        say("  %s" % ps)
        g.build(reads, offs, rs.k)  # statistics add up over builds
        ps2 = g.probe_stats()
        assert ps2["lookups"] == 2 * ps["lookups"], (ps, ps2)
        assert ps2["cas_attempts"] - ps2["cas_lost"] == V, ps2  # no new vertex in the second build
        g.reset()
        assert g.probe_stats()["lookups"] == 0
    with dbg.Graph(expected_vertices=V, flags=mode) as g:  # without the flag: zeros
        g.build(reads, offs, rs.k)
        assert g.probe_stats()["lookups"] == 0
