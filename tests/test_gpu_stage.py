"""Partition scatter shapes (dbg_config bin_shape1 / bin_shape2) through the
C ABI: plain tiles, staged lines (each run's records wait in LDS until they
fill a 128-byte line; only whole lines are stored) and big tiles of 16384
records.  The graph must not depend on the shape: every shape of either
scatter builds the oracle's graph, with one-word and two-word records, on
inputs whose chunks end in partial lines and partial big tiles, and the
graph reports the shapes it used (dbg_stats bin_shape1 / bin_shape2)."""

import numpy as np
import pytest

import oracle
import readsim
import records
import paper_2401_02756_amd as dbg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

T, S, B, BW = dbg.SHAPE_TILES, dbg.SHAPE_STAGED, dbg.SHAPE_BIG, dbg.SHAPE_BIG_WIDE


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def say(msg):
    print("[case] " + msg, flush=True)


def _inputs():
    tiny = readsim.make_config(1)
    bac = readsim.make_config(2)
    n = 150_000
    cut = readsim.ReadSet(reads=bac.reads[:int(bac.offsets[n])], offsets=bac.offsets[:n + 1], k=bac.k)
    return [("tiny", tiny), ("bacterial slice", cut)]


# requested shapes -> shapes used on these small tables (automatic: big tiles for both
# scatters of one-word records, 8192 records in the first below 385 runs; for two-word records
# plain tiles in the first below 385 runs).  Wide big tiles (16384 one-word records) exist in the
# first scatter only: requested for the second, it takes big tiles (128 KB already).
CASES = [((0, 0), (B, B)), ((T, T), (T, T)), ((S, S), (S, S)), ((B, B), (B, B)), ((B, S), (B, S)),
         ((S, B), (S, B)), ((BW, BW), (BW, B)), ((BW, S), (BW, S))]


@pytest.mark.parametrize("req,used", CASES, ids=["auto", "tiles", "staged", "big", "big-staged", "staged-big",
                                                 "wide", "wide-staged"])
def test_shapes_build_the_oracle_graph(req, used):
    for name, rs in _inputs():
        ref = oracle.build_graph(rs.reads, rs.offsets, rs.k)
        for chunks in (0, 4, 64):  # default chunks, fewer (longer), more (down to big tiles' minimum)
            say("%s, shapes %s, bin_chunks %d" % (name, req, chunks))
            with dbg.Graph(expected_vertices=ref[0].shape[0], load_factor=0.5, flags=dbg.F_BINNED,
                           bin_shape1=req[0], bin_shape2=req[1], bin_chunks=chunks) as g:
                g.build(rs.reads, rs.offsets, rs.k)
                st = g.stats()
                assert (st["bin_shape1"], st["bin_shape2"]) == used, st
                records.assert_exact(ref, g.extract(), "%s, shapes %s" % (name, req))


def test_shapes_long_keys():
    """Two-word records (k = 45): 16-byte records, eight to a line; big
    tiles hold 8192 of them (the same 128 KB of LDS)."""
    rng = np.random.default_rng(11)
    k = 45
    reads = ["".join("ACGT"[x] for x in rng.integers(0, 4, int(rng.integers(40, 300)))) for _ in range(3000)]
    rs = readsim.reads_from_strings(reads, k)
    hi, lo, c = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    for req, used in (((T, T), (T, T)), ((S, S), (S, S)), ((B, B), (B, B)), ((0, 0), (T, B)), ((BW, BW), (B, B))):
        say("long k, shapes %s: %d vertices" % (req, hi.shape[0]))
        with dbg.Graph(expected_vertices=hi.shape[0], flags=dbg.F_BINNED, bin_shape1=req[0],
                       bin_shape2=req[1]) as g:
            g.build(rs.reads, rs.offsets, k)
            st = g.stats()
            assert (st["bin_shape1"], st["bin_shape2"]) == used, st
            keys, counts = g.extract_sorted()
        assert np.array_equal(keys[:, 0], hi) and np.array_equal(keys[:, 1], lo) and np.array_equal(counts, c)


@pytest.mark.parametrize("req", [(S, S), (B, S), (B, B), (BW, B)], ids=["staged", "big-staged", "big", "wide"])
def test_shapes_device_graph_and_batch(req):
    """Shaped scatters under graph capture (replayed) and in a batched pass."""
    sets = [readsim.simulate(int(gl), 120, 12.0, 0.01, 31, seed=500 + j) for j, gl in enumerate((3000, 20000, 9000))]
    refs = [oracle.build_graph(x.reads, x.offsets, x.k) for x in sets]
    x = sets[1]
    d_reads = torch.from_numpy(x.reads).cuda()
    d_off = torch.from_numpy(x.offsets.astype(np.int64)).cuda()
    with dbg.Graph(expected_vertices=refs[1][0].shape[0], flags=dbg.F_BINNED | dbg.F_GRAPH, bin_shape1=req[0],
                   bin_shape2=req[1]) as g:
        for rep in range(3):
            say("captured pass, shapes %s, replay %d" % (req, rep))
            g.reset()
            g.build_device(d_reads, d_off, x.k)
            g.sync()
            records.assert_exact(refs[1], g.extract(), "replay %d" % rep)
        st = g.stats()
        assert st["graph_replays"] >= 2 and (st["bin_shape1"], st["bin_shape2"]) == req
    gs = [dbg.Graph(expected_vertices=r[0].shape[0], flags=dbg.F_BINNED, bin_shape1=req[0], bin_shape2=req[1])
          for r in refs]
    try:
        say("batched pass, shapes %s, %d sets" % (req, len(sets)))
        assert dbg.build_batch(gs, [(s.reads, s.offsets, s.k) for s in sets]) == [0] * len(sets)
        for j, (g, r) in enumerate(zip(gs, refs)):
            records.assert_exact(r, g.extract(), "set %d" % j)
    finally:
        for g in gs:
            g.close()
