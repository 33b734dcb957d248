"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
worked example and letter code, brute force by sorting strings, a closed form
for error-free reads, the Eulerian path of a single read, and invariants.  The
mutation tests plant mistakes in oracle output and check that the pins catch
them.
"""

import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import readsim
from oracle import brute, euler, invariants
from conftest import read_golden

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def build_strings(reads, k):
    rs = readsim.reads_from_strings(reads, k)
    return oracle.build_graph(rs.reads, rs.offsets, k), rs


# ---------------------------------------------------------------- paper pins

def test_letter_code_matches_paper():
    table = {r[0]: int(r[1]) for r in read_golden("letter_code.txt")}
    for ch, code in table.items():
        # as a vertex: the single-letter (k-1)-mer has key = code
        (keys, counts), _ = build_strings([ch + "A"], 2)
        assert keys.tolist() == sorted({code, 0})
        # as an edge letter: vertex A gets its counter `code` raised
        (keys, counts), _ = build_strings(["A" + ch], 2)
        row = counts[keys.tolist().index(0)]
        assert row.tolist() == [1 if i == code else 0 for i in range(4)]


def test_worked_example_oracle(worked_example):
    read, k, verts = worked_example
    (keys, counts), _ = build_strings([read], k)
    got = {oracle.decode_key(x, k): (int(x), c.tolist()) for x, c in zip(keys, counts)}
    assert got == verts
    # the vertex set printed in the paper
    assert set(got) == {"ACG", "CGC", "CGA", "GAC"}


def test_worked_example_brute(worked_example):
    read, k, verts = worked_example
    g = brute.brute_graph([read], k)
    want = {v: {oracle.LETTERS[i]: c for i, c in enumerate(cs) if c} for v, (_, cs) in verts.items()}
    assert g == want


def test_worked_example_eulerian_path(worked_example):
    read, k, _ = worked_example
    (keys, counts), _ = build_strings([read], k)
    assert euler.eulerian_spelling(keys, counts, k) == read


# ---------------------------------------------------------------- brute force

alphabet = st.sampled_from(["AC", "ACGT", "acgt", "AT", "G", "ACgT"])


@settings(max_examples=150, deadline=None)
@given(data=st.data(), k=st.integers(2, 8))
def test_oracle_matches_brute_force(data, k):
    letters = data.draw(alphabet)
    nreads = data.draw(st.integers(0, 6))
    reads = [data.draw(st.text(alphabet=letters, min_size=0, max_size=30)) for _ in range(nreads)]
    (keys, counts), rs = build_strings(reads, k)
    assert oracle.graph_to_dict(keys, counts, k) == brute.brute_graph(reads, k)
    if len(keys):
        invariants.check_graph(keys, counts, rs.reads, rs.offsets, k)


def test_short_reads_edge_cases():
    k = 5
    # length k-1: no k-mer, no vertex; length k: two vertices, one edge
    (keys, counts), _ = build_strings(["ACGT"], k)
    assert keys.size == 0
    (keys, counts), _ = build_strings(["ACGTA"], k)
    assert [oracle.decode_key(x, k) for x in keys] == ["ACGT", "CGTA"] or \
        sorted(oracle.decode_key(x, k) for x in keys) == ["ACGT", "CGTA"]
    assert int(counts.sum()) == 1
    (keys, counts), _ = build_strings([], k)
    assert keys.size == 0
    (keys, counts), _ = build_strings(["", "AC", "GGGGGG"], k)
    assert [oracle.decode_key(x, k) for x in keys] == ["GGGG"]
    assert counts.tolist() == [[0, 0, 0, 2]]


def test_k_bounds_and_validation():
    rs = readsim.reads_from_strings(["ACGTACGT"], 4)
    for bad_k in (0, 1, 33, 64):
        with pytest.raises(oracle.OracleError) as e:
            oracle.build_graph(rs.reads, rs.offsets, bad_k)
        assert e.value.code == oracle.E_K
    bad = readsim.reads_from_strings(["ACGTNACGT"], 4)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_graph(bad.reads, bad.offsets, 4)
    assert e.value.code == oracle.E_BASE
    off = np.array([0, 5, 3, 8], dtype=np.uint64)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_graph(rs.reads, off, 4)
    assert e.value.code == oracle.E_INVAL


def test_k32_uses_all_62_bits():
    rng = random.Random(7)
    read = "".join(rng.choice("ACGT") for _ in range(80))
    (keys, counts), rs = build_strings([read, read.lower()], 32)
    assert oracle.graph_to_dict(keys, counts, 32) == brute.brute_graph([read, read.lower()], 32)
    assert int(keys.max()) < (1 << 62)
    invariants.check_graph(keys, counts, rs.reads, rs.offsets, 32)


# ---------------------------------------------------------------- closed form

def closed_form(genome: str, starts, L: int, k: int):
    """Counts of error-free reads from a genome whose (k-1)-mers are distinct:
    the k-mer at genome position p is covered by every read with start s in
    [p - (L - k), p]; vertices are the windows at covered positions."""
    G = len(genome)
    diff = np.zeros(G + 1, dtype=np.int64)
    for s in starts:
        diff[s] += 1
        diff[s + L - k + 1] -= 1
    edge_cov = np.cumsum(diff)[:G]          # reads covering k-mer at p
    vdiff = np.zeros(G + 2, dtype=np.int64)
    for s in starts:
        vdiff[s] += 1
        vdiff[s + L - k + 2] -= 1
    vert_cov = np.cumsum(vdiff)[:G + 1]
    out = {}
    for p in range(G - k + 2):
        if vert_cov[p] > 0:
            out[genome[p:p + k - 1]] = {}
    for p in range(G - k + 1):
        if edge_cov[p] > 0:
            out[genome[p:p + k - 1]][genome[p + k - 1]] = int(edge_cov[p])
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_closed_form_error_free(seed):
    k, L = 17, 60
    rs = readsim.simulate(3000, L, 8.0, 0.0, k, seed, keep_genome=True)
    genome = rs.genome.tobytes().decode()
    assert len({genome[p:p + k - 1] for p in range(len(genome) - k + 2)}) == len(genome) - k + 2
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, k)
    assert oracle.graph_to_dict(keys, counts, k) == closed_form(genome, rs.starts, L, k)


# ---------------------------------------------------------------- Eulerian path

@pytest.mark.parametrize("seed", range(5))
def test_single_read_eulerian_path(seed):
    rng = random.Random(seed)
    k = 15
    while True:
        read = "".join(rng.choice("ACGT") for _ in range(200))
        wins = [read[j:j + k - 1] for j in range(len(read) - k + 2)]
        if len(set(wins)) == len(wins):
            break
    (keys, counts), rs = build_strings([read], k)
    assert euler.eulerian_spelling(keys, counts, k) == read


# ---------------------------------------------------------------- cross-checks

def test_oracle_matches_sort_build_config1():
    rs = readsim.make_config(1)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    sk, sc = invariants.sort_build(rs.reads, rs.offsets, rs.k)
    assert np.array_equal(keys, sk)
    assert np.array_equal(counts, sc)
    invariants.check_graph(keys, counts, rs.reads, rs.offsets, rs.k)
    assert 15_000 < keys.shape[0] < 21_000


def test_oracle_matches_sort_build_scaled_config2():
    rs = readsim.make_config(2, scale=0.02)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    sk, sc = invariants.sort_build(rs.reads, rs.offsets, rs.k)
    assert np.array_equal(keys, sk)
    assert np.array_equal(counts, sc)
    invariants.check_graph(keys, counts, rs.reads, rs.offsets, rs.k)


def test_partitions_union_is_the_whole():
    rs = readsim.make_config(1)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    parts = [oracle.build_graph(rs.reads, rs.offsets, rs.k, 5, p) for p in range(5)]
    uk = np.concatenate([p[0] for p in parts])
    uc = np.concatenate([p[1] for p in parts])
    order = np.argsort(uk)
    assert np.array_equal(uk[order], keys)
    assert np.array_equal(uc[order], counts)
    for p, (pk, _) in enumerate(parts):
        assert np.all(oracle.partition_of(pk, 5) == p)


def test_chunked_and_parallel_builds_equal_the_plain_one():
    rs = readsim.make_config(2, scale=0.01)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    for chunks in (2, 7):
        ck, cc = oracle.build_graph_chunked(rs.reads, rs.offsets, rs.k, chunks=chunks)
        assert np.array_equal(ck, keys) and np.array_equal(cc, counts)
    pk, pc = oracle.build_graph(rs.reads, rs.offsets, rs.k, 16, 3)
    ck, cc = oracle.build_graph_chunked(rs.reads, rs.offsets, rs.k, 16, 3, chunks=5)
    assert np.array_equal(ck, pk) and np.array_equal(cc, pc)
    qk, qc = oracle.build_graph_parallel(rs.reads, rs.offsets, rs.k, threads=4)
    assert np.array_equal(qk, keys) and np.array_equal(qc, counts)


def test_vertex_counts_one_by_one():
    rs = readsim.make_config(1)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    rng = np.random.default_rng(0)
    for i in rng.choice(keys.shape[0], 20, replace=False):
        seen, c = oracle.vertex_counts(rs.reads, rs.offsets, rs.k, int(keys[i]))
        assert seen and np.array_equal(c, counts[i])
    seen, c = oracle.vertex_counts(rs.reads, rs.offsets, rs.k, int(keys.max()) + 1)
    assert not seen or int(keys.max()) + 1 in set(keys.tolist())


def test_read_order_and_splitting_invariance():
    rs = readsim.make_config(1)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    L = rs.lengths()
    perm = np.random.default_rng(3).permutation(rs.n_reads)
    reads2 = [rs.read(i) for i in perm]
    rs2 = readsim.reads_from_strings(reads2, rs.k)
    k2, c2 = oracle.build_graph(rs2.reads, rs2.offsets, rs.k)
    assert np.array_equal(keys, k2) and np.array_equal(counts, c2)
    # two halves built separately, then merged by key
    h = rs.n_reads // 2
    a = readsim.reads_from_strings([rs.read(i) for i in range(h)], rs.k)
    b = readsim.reads_from_strings([rs.read(i) for i in range(h, rs.n_reads)], rs.k)
    ka, ca = oracle.build_graph(a.reads, a.offsets, rs.k)
    kb, cb = oracle.build_graph(b.reads, b.offsets, rs.k)
    mk = np.union1d(ka, kb)
    mc = np.zeros((mk.shape[0], 4), dtype=np.uint32)
    mc[np.searchsorted(mk, ka)] += ca
    mc[np.searchsorted(mk, kb)] += cb
    assert np.array_equal(mk, keys) and np.array_equal(mc, counts)
    assert L.sum() == rs.total_bases


def test_paper_8bit_counters_would_wrap():
    """The paper keeps 8-bit counters and says 255 is enough (Methods, "Graph
    data structure").  With a 1 kbp unit repeated 50 times at 30x, one edge is
    seen far more often, so the build keeps 32-bit counters."""
    G, L, k = 200_000, 150, 31
    rs = readsim.simulate(G, L, 30.0, 0.01, k, 11, repeats=[(0, 1000)] * 50)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, k)
    assert int(counts.max()) > 255
    assert int(counts.sum()) == invariants.expected_total(rs.offsets, k)


# ---------------------------------------------------------------- planted mistakes

def _mutants(keys, counts, k):
    """Plausible mistakes in an oracle's output, one at a time."""
    V = keys.shape[0]
    sink = int(np.nonzero(counts.sum(axis=1) == 0)[0][0])
    busy = int(np.argmax(counts.sum(axis=1)))
    yield "dropped sink vertex", np.delete(keys, sink), np.delete(counts, sink, axis=0)
    ac = int(np.nonzero(counts[:, 0] != counts[:, 1])[0][0])
    c = counts.copy(); c[ac] = c[ac][[1, 0, 2, 3]]
    yield "swapped letters A/C", keys, c
    tg = int(np.nonzero(counts[:, 2] != counts[:, 3])[0][0])
    c = counts.copy(); c[tg] = c[tg][[0, 1, 3, 2]]
    yield "swapped letters T/G (alphabetical order)", keys, c
    c = counts.copy(); nz = np.nonzero(c[busy])[0][0]; c[busy, nz] -= 1
    yield "dropped one k-mer", keys, c
    c = counts.copy(); nz = np.nonzero(c[busy])[0][0]; c[busy, nz] -= 1; c[(busy + 1) % V, nz] += 1
    yield "count on the wrong vertex", keys, c
    mask = (1 << (2 * (k - 1))) - 1
    rev = np.array([int(format(int(x), "0%db" % (2 * (k - 1)))[::-1], 2) & mask for x in keys],
                   dtype=np.uint64)
    yield "bit-reversed keys", rev, counts


def test_invariants_catch_planted_mistakes():
    rs = readsim.make_config(1)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    invariants.check_graph(keys, counts, rs.reads, rs.offsets, rs.k)
    for name, mk, mc in _mutants(keys, counts, rs.k):
        with pytest.raises(AssertionError):
            invariants.check_graph(mk, mc, rs.reads, rs.offsets, rs.k)


def test_worked_example_catches_reversed_key_order(worked_example):
    read, k, verts = worked_example
    # LSB-first packing would give ACG -> 0b110100 = 52, not the MSB-first 7
    assert verts["ACG"][0] == 7 and verts["GAC"][0] == 49
