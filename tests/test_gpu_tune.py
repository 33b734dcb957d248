"""The autotuner through the C ABI: it picks a valid configuration, caches it
in the process and in its cache file, the graph built with its choice is
bit-identical to the oracle's, and so is the graph built under every
configuration of its search space."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import readsim
import records
import paper_2401_02756_amd as dbg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

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


def same(got, want, what):
    assert got[0].shape == want[0].shape, what
    assert np.array_equal(got[0], want[0]), what + ": keys"
    assert np.array_equal(got[1], want[1]), what + ": counts"


def on_device(rs):
    return (torch.from_numpy(rs.reads).cuda(), torch.from_numpy(rs.offsets.astype(np.int64)).cuda())


def check_choice(t):
    assert 0.3 <= t.load_factor <= 0.75
    assert t.flags & ~(dbg.F_BINNED | dbg.F_MERGE) == 0
    if t.flags & dbg.F_BINNED:
        assert t.block_size == 0 and t.windows_per_thread == 0 and not t.flags & dbg.F_MERGE
        assert t.bin_chunks in (0, 4, 8, 16, 64) and t.bin_scatter_div in (0, 1, 2, 4) and (t.bin_shape1, t.bin_shape2) in (
            (0, 0), (1, 1), (2, 2), (3, 3), (3, 2), (4, 3))
    else:
        assert t.block_size in (256, 512, 1024) and t.windows_per_thread in (2, 4, 8)
        assert t.bin_chunks == 0 and t.bin_scatter_div == 0 and t.bin_shape1 == 0 and t.bin_shape2 == 0
    assert t.best_ms > 0


@pytest.mark.parametrize("k", [21, 32])
def test_autotune_plain(k):
    rs = readsim.simulate(40_000, 150, 20.0, 0.01, k, seed=77)
    ev = readsim.expected_vertices(40_000, 150, rs.n_reads, 0.01, k)
    d_reads, d_off = on_device(rs)
    say("plain k=%d, %d reads" % (k, rs.n_reads))
    t = dbg.autotune([0, rs.n_reads], [k], d_reads, d_off, [ev], keep_flags=dbg.F_GRAPH, force=True)
    check_choice(t)
    assert t.from_cache == 0 and t.candidates >= 4
    if k == 32:
        assert not t.flags & dbg.F_BINNED  # binned records hold k <= 31
    again = dbg.autotune([0, rs.n_reads], [k], d_reads, d_off, [ev], keep_flags=dbg.F_GRAPH)
    assert again.from_cache == 1 and again.candidates == 0
    assert (again.flags, again.load_factor, again.block_size) == (t.flags, t.load_factor, t.block_size)
    kw = t.graph_kwargs()
    kw["flags"] |= dbg.F_GRAPH
    with dbg.Graph(expected_vertices=ev, **kw) as g:
        g.build_device(d_reads, d_off, k)
        g.sync()
        same(g.extract_sorted(), oracle.build_graph(rs.reads, rs.offsets, k), "tuned plain build")


def test_autotune_batch():
    sets = [readsim.simulate(int(g), 100, 15.0, 0.008, k, seed=300 + j)
            for j, (g, k) in enumerate([(5000, 21), (30000, 31), (12000, 21), (60000, 31),
                                        (2000, 31), (25000, 21)])]
    ev = [readsim.expected_vertices(rs.meta["genome_len"], 100, rs.n_reads, 0.008, rs.k) for rs in sets]
    reads = np.concatenate([rs.reads for rs in sets])
    lens = np.concatenate([rs.lengths() for rs in sets])
    off = np.zeros(lens.shape[0] + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    rb = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([rs.n_reads for rs in sets], out=rb[1:])
    ks = [rs.k for rs in sets]
    d_reads, d_off = torch.from_numpy(reads).cuda(), torch.from_numpy(off).cuda()
    say("batched, %d instances" % len(sets))
    t = dbg.autotune(rb, ks, d_reads, d_off, ev, force=True)
    check_choice(t)
    gs = [dbg.Graph(expected_vertices=e, **t.graph_kwargs()) for e in ev]
    try:
        assert dbg.build_batch_device(gs, rb, ks, d_reads, d_off) == [0] * len(sets)
        for j, (g, rs) in enumerate(zip(gs, sets)):
            same(g.extract_sorted(), oracle.build_graph(rs.reads, rs.offsets, rs.k), "instance %d" % j)
    finally:
        for g in gs:
            g.close()


def test_every_configuration_builds_the_oracle_graph():
    """Every configuration the tuner may time (dbg_autotune_space) builds the
    oracle's graph, on the tiny workload and on a slice of the bacterial one."""
    tiny = readsim.make_config(1)
    bac = readsim.make_config(2)
    n = 20_000
    cut = readsim.ReadSet(reads=bac.reads[:int(bac.offsets[n])], offsets=bac.offsets[:n + 1], k=bac.k)
    inputs = []
    for name, rs in (("tiny", tiny), ("bacterial slice", cut)):
        want = oracle.build_graph(rs.reads, rs.offsets, rs.k)
        inputs.append((name, rs, want) + on_device(rs))
    space = [(True, c) for c in dbg.autotune_space(True)] + [(False, c) for c in dbg.autotune_space(False)]
    say("%d configurations x %d inputs" % (len(space), len(inputs)))
    for binned, c in space:
        for name, rs, want, d_reads, d_off in inputs:
            kw = c.graph_kwargs()
            with dbg.Graph(expected_vertices=want[0].shape[0], **kw) as g:
                g.build_device(d_reads, d_off, rs.k)
                g.sync()
                records.assert_exact(want, g.extract(), "%s, %s" % (name, json.dumps(c.as_dict())))


_TUNE_CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import readsim
import paper_2401_02756_amd as dbg
rs = readsim.make_config(1)
d_reads = torch.from_numpy(rs.reads).cuda()
d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
t = dbg.autotune([0, rs.n_reads], [rs.k], d_reads, d_off, [rs.meta["expected_vertices"]])
print(json.dumps(t.as_dict()))
"""


def test_tuning_persists_in_the_cache_file(tmp_path):
    """A tuning is written to the cache file; a later process reads it
    instead of searching again."""
    path = tmp_path / "autotune.tsv"
    env = dict(os.environ, DBG_TUNE_CACHE=str(path))
    runs = []
    for i in range(2):
        say("tuning process %d" % i)
        out = subprocess.run([sys.executable, "-c", _TUNE_CHILD, ROOT], env=env, capture_output=True, text=True,
                             timeout=240, cwd=ROOT)
        assert out.returncode == 0, out.stderr[-2000:]
        runs.append(json.loads(out.stdout.strip().splitlines()[-1]))
    first, second = runs
    assert first["from_cache"] == 0 and first["candidates"] >= 4
    assert second["from_cache"] == 2 and second["candidates"] == 0
    for key in ("load_factor", "flags", "block_size", "windows_per_thread", "bin_chunks", "bin_scatter_div",
                "bin_shape1", "bin_shape2"):
        assert first[key] == second[key], key
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and "\t" in lines[0] and "gfx" in lines[0]
