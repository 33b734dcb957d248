"""Line-staged partition scatters (dbg_config bin_stage) through the C ABI.

A staged scatter keeps each run's records in LDS until they fill a 128-byte
line and stores whole lines; the graph must not depend on it.  Every staging
mode builds the oracle's graph, with one-word and two-word records, on
inputs whose chunks end in partial lines, and the graph reports which
scatters staged (dbg_stats bin_staged)."""

import numpy as np
import pytest

import oracle
import readsim
import records
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


def _inputs():
    tiny = readsim.make_config(1)
    bac = readsim.make_config(2)
    n = 150_000
    cut = readsim.ReadSet(reads=bac.reads[:int(bac.offsets[n])], offsets=bac.offsets[:n + 1], k=bac.k)
    return [("tiny", tiny), ("bacterial slice", cut)]


@pytest.mark.parametrize("stage,want", [(0, 0), (1, 0), (2, 3)])
def test_staging_modes_build_the_oracle_graph(stage, want):
    for name, rs in _inputs():
        ref = oracle.build_graph(rs.reads, rs.offsets, rs.k)
        for chunks in (0, 4):  # default chunks, and 4 per workgroup (longer chunks, fewer partial lines)
            say("%s, bin_stage %d, bin_chunks %d" % (name, stage, chunks))
            with dbg.Graph(expected_vertices=ref[0].shape[0], load_factor=0.5, flags=dbg.F_BINNED,
                           bin_stage=stage, bin_chunks=chunks) as g:
                g.build(rs.reads, rs.offsets, rs.k)
                st = g.stats()
                # a small table: buckets span few segments, so only bin_stage 2 stages
                assert st["bin_stage"] == stage and st["bin_staged"] == want, st
                records.assert_exact(ref, g.extract(), "%s, stage %d" % (name, stage))


def test_staged_long_keys():
    """Two-word records (k = 45): 16-byte records, eight to a line."""
    rng = np.random.default_rng(11)
    k = 45
    reads = ["".join("ACGT"[x] for x in rng.integers(0, 4, int(rng.integers(40, 300)))) for _ in range(3000)]
    rs = readsim.reads_from_strings(reads, k)
    hi, lo, c = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    for stage in (1, 2):
        say("long k, bin_stage %d: %d vertices" % (stage, hi.shape[0]))
        with dbg.Graph(expected_vertices=hi.shape[0], flags=dbg.F_BINNED, bin_stage=stage) as g:
            g.build(rs.reads, rs.offsets, k)
            assert g.stats()["bin_staged"] == (3 if stage == 2 else 0)
            keys, counts = g.extract_sorted()
        assert np.array_equal(keys[:, 0], hi) and np.array_equal(keys[:, 1], lo) and np.array_equal(counts, c)


def test_staged_device_graph_and_batch():
    """Staged scatters under graph capture (replayed) and in a batched pass."""
    sets = [readsim.simulate(int(gl), 120, 12.0, 0.01, 31, seed=500 + j) for j, gl in enumerate((3000, 20000, 9000))]
    refs = [oracle.build_graph(x.reads, x.offsets, x.k) for x in sets]
    x = sets[1]
    d_reads = torch.from_numpy(x.reads).cuda()
    d_off = torch.from_numpy(x.offsets.astype(np.int64)).cuda()
    with dbg.Graph(expected_vertices=refs[1][0].shape[0], flags=dbg.F_BINNED | dbg.F_GRAPH, bin_stage=2) as g:
        for rep in range(3):
            say("captured staged pass, replay %d" % rep)
            g.reset()
            g.build_device(d_reads, d_off, x.k)
            g.sync()
            records.assert_exact(refs[1], g.extract(), "replay %d" % rep)
        assert g.stats()["graph_replays"] >= 2 and g.stats()["bin_staged"] == 3
    gs = [dbg.Graph(expected_vertices=r[0].shape[0], flags=dbg.F_BINNED, bin_stage=2) for r in refs]
    try:
        say("batched staged pass, %d sets" % len(sets))
        assert dbg.build_batch(gs, [(s.reads, s.offsets, s.k) for s in sets]) == [0] * len(sets)
        for j, (g, r) in enumerate(zip(gs, refs)):
            records.assert_exact(r, g.extract(), "set %d" % j)
    finally:
        for g in gs:
            g.close()
