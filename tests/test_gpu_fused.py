"""dbg_build_extract_device: a build whose graph comes out in the same call.

For a binned graph (k <= 31, or 33 <= k <= 63 with two-word keys) the
vertices are written by the build's reduce kernel, one reserved range per
table segment; otherwise the call builds and then extracts.  Either way the records, sorted, must equal the
oracle's graph over every build of the handle, bit for bit.
"""

import dataclasses

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


def dev(rs):
    return torch.from_numpy(rs.reads).cuda(), torch.from_numpy(rs.offsets.astype(np.int64)).cuda()


def out_buffers(cap, kw=1):
    keys = torch.full((cap * kw,), -1, dtype=torch.int64, device="cuda")
    counts = torch.full((cap, 4), -1, dtype=torch.int32, device="cuda")
    return keys, counts


def host_sorted(keys, counts, n, kw=1):
    k = keys.cpu().numpy().view(np.uint64)[: n * kw]
    c = counts.cpu().numpy().view(np.uint32)[:n]
    if kw == 2:
        k = k.reshape(n, 2)
        order = np.lexsort((k[:, 1], k[:, 0]))
    else:
        order = np.argsort(k, kind="stable")
    return k[order], c[order]


def assert_same(got, want, what):
    assert got[0].shape == want[0].shape, "%s: %d vertices, oracle has %d" % (what, got[0].shape[0],
                                                                             want[0].shape[0])
    assert np.array_equal(got[0], want[0]), "%s: keys differ" % what
    assert np.array_equal(got[1], want[1]), "%s: counts differ" % what


def fused(g, rs, cap, kw=1):
    d_reads, d_off = dev(rs)
    keys, counts = out_buffers(cap, kw)
    n = g.build_extract_device(d_reads, d_off, rs.k, keys, counts)
    return host_sorted(keys, counts, n, kw), n


@pytest.mark.parametrize("lf", [0.4, 0.85])
def test_fused_binned_matches_oracle(lf):
    rs = readsim.make_config(1)
    say("fused binned build, configuration 1, load factor %.2f" % lf)
    want = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    with dbg.Graph(load_factor=lf, flags=dbg.F_BINNED) as g:
        got, n = fused(g, rs, want[0].shape[0] + 17)
        assert n == want[0].shape[0] == g.vertex_count()
        assert_same(got, want, "fused output")
        assert_same(g.extract_sorted(), want, "extraction after the fused build")


def test_fused_scaled_bacterial():
    rs = readsim.make_config(2, scale=0.1)
    say("fused binned build, bacterial reads at 0.1 scale")
    want = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    with dbg.Graph(expected_vertices=rs.meta["expected_vertices"], load_factor=0.4, flags=dbg.F_BINNED) as g:
        got, n = fused(g, rs, g.stats()["capacity"])
        assert_same(got, want, "fused output")


def test_fused_accumulates_and_reports_space():
    rs = readsim.make_config(1)
    say("fused builds accumulate; a short output buffer gives DBG_E_SPACE")
    wk, wc = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    V = wk.shape[0]
    with dbg.Graph(flags=dbg.F_BINNED) as g:
        g.build(rs.reads, rs.offsets, rs.k)
        got, n = fused(g, rs, V)  # second build: every count doubles, old vertices come out too
        assert n == V
        assert_same(got, (wk, 2 * wc), "second build")
        d_reads, d_off = dev(rs)
        keys, counts = out_buffers(V - 1)
        with pytest.raises(dbg.DbgError) as e:
            g.build_extract_device(d_reads, d_off, rs.k, keys, counts)
        assert e.value.code == dbg.E_SPACE
        assert g.vertex_count() == V  # the build itself went through
        assert_same(g.extract_sorted(), (wk, 3 * wc), "after DBG_E_SPACE")
        # no reads: the call only extracts; no output buffer: only the count
        keys, counts = out_buffers(V)
        e_reads = torch.empty(0, dtype=torch.uint8, device="cuda")
        e_off = torch.zeros(1, dtype=torch.int64, device="cuda")
        n = g.build_extract_device(e_reads, e_off, rs.k, keys, counts)
        assert_same(host_sorted(keys, counts, n), (wk, 3 * wc), "empty input")
        assert g.build_extract_device(e_reads, e_off, rs.k, None, None) == V


@pytest.mark.parametrize("k", [33, 45, 63])
def test_fused_long_k_matches_oracle(k):
    rs = readsim.make_config(1)
    say("fused binned build of two-word keys, k = %d" % k)
    hi, lo, wc = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    with dbg.Graph(load_factor=0.5, flags=dbg.F_BINNED) as g:
        got, n = fused(g, dataclasses.replace(rs, k=k), hi.shape[0] + 5, kw=2)
        assert g.stats()["binned"] == 1 and n == hi.shape[0]
    assert_same(got, (np.stack([hi, lo], axis=1), wc), "fused output, k = %d" % k)


@pytest.mark.parametrize("flags,k", [(0, 21), (dbg.F_MERGE, 31), (dbg.F_BINNED, 32), (dbg.F_BINNED, 45),
                                     (0, 51)])
def test_other_modes_equal_extract(flags, k):
    rs = readsim.make_config(1)
    say("build_extract_device vs dbg_extract: flags %d, k = %d" % (flags, k))
    kw = 2 if k > 32 else 1
    with dbg.Graph(load_factor=0.5, flags=flags) as g:
        d_reads, d_off = dev(rs)
        keys, counts = out_buffers(60_000, kw)
        n = g.build_extract_device(d_reads, d_off, k, keys, counts)
        got = host_sorted(keys, counts, n, kw)
        assert_same(got, g.extract_sorted(), "same graph as dbg_extract")
    if k <= 32:
        assert_same(got, oracle.build_graph(rs.reads, rs.offsets, k), "oracle")


def test_fused_captured_replays_take_new_buffers():
    say("captured passes: fused calls into alternating buffers, plain builds in between")
    sets = [readsim.simulate(genome_len=40_000, read_len=100, coverage=15.0, err=0.005, k=21, seed=77 + j)
            for j in range(3)]
    wants = [oracle.build_graph(s.reads, s.offsets, s.k) for s in sets]
    vmax = max(w[0].shape[0] for w in wants)
    bufs = [out_buffers(vmax), out_buffers(vmax)]
    with dbg.Graph(expected_vertices=vmax, flags=dbg.F_BINNED | dbg.F_GRAPH) as g:
        for rnd in range(6):
            j = rnd % 3
            rs = sets[j]
            g.reset()
            d_reads, d_off = dev(rs)
            if rnd == 3:  # a plain captured build: its pass must leave the output buffers alone
                g.build_device(d_reads, d_off, rs.k)
                g.sync()
                assert_same(g.extract_sorted(), wants[j], "plain build, round %d" % rnd)
                keys, counts = bufs[0]  # round 2's output
                assert_same(host_sorted(keys, counts, last_n), wants[2], "round 2 output after round 3")
                continue
            keys, counts = bufs[rnd % 2]
            keys.fill_(-1)
            n = g.build_extract_device(d_reads, d_off, rs.k, keys, counts)
            assert_same(host_sorted(keys, counts, n), wants[j], "fused replay, round %d" % rnd)
            last_n = n
        assert g.stats()["graph_replays"] > 0
