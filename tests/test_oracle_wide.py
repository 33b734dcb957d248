"""Pins of the oracle's long-k build (k up to 64, keys of up to 126 bits).

The wide build packs each window into a 128-bit integer from scratch and keeps
its own map, so it is checked against things it shares nothing with: string
brute force, the 64-bit build where both apply, the closed form of error-free
reads, the Eulerian path of a single read, and the bit budget of k = 64.
"""

import random

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import readsim
from oracle import brute

from test_oracle import closed_form

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def wide_dict(hi, lo, counts, k):
    out = {}
    for h, l, c in zip(hi.tolist(), lo.tolist(), counts.tolist()):
        out[oracle.decode_wide_key(h, l, k)] = {oracle.LETTERS[i]: int(c[i]) for i in range(4) if c[i]}
    return out


def build(reads, k):
    rs = readsim.reads_from_strings(reads, k)
    return oracle.build_graph_wide(rs.reads, rs.offsets, k)


@pytest.mark.parametrize("k", [2, 3, 9, 21, 31, 32])
def test_short_k_equals_the_64bit_build(k):
    rs = readsim.simulate(4000, 90, 6.0, 0.01, k, 40 + k)
    hi, lo, counts = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    keys, want = oracle.build_graph(rs.reads, rs.offsets, k)
    assert not hi.any()
    assert np.array_equal(lo, keys) and np.array_equal(counts, want)


@settings(max_examples=120, deadline=None)
@given(data=st.data(), k=st.integers(33, 64))
def test_matches_brute_force(data, k):
    letters = data.draw(st.sampled_from(["AC", "ACGT", "acgt", "G", "ACgT"]))
    nreads = data.draw(st.integers(0, 5))
    reads = [data.draw(st.text(alphabet=letters, min_size=0, max_size=110)) for _ in range(nreads)]
    assert wide_dict(*build(reads, k), k) == brute.brute_graph(reads, k)


def test_order_is_numeric_on_the_full_key():
    # keys that differ only in the high word, and only in the low word
    rng = random.Random(3)
    reads = ["".join(rng.choice("ACGT") for _ in range(120)) for _ in range(30)]
    hi, lo, _ = build(reads, 51)
    full = [(int(h) << 64) | int(l) for h, l in zip(hi, lo)]
    assert full == sorted(full) and len(set(full)) == len(full)
    assert len(set(hi.tolist())) > 1


@pytest.mark.parametrize("k", [33, 51, 64])
def test_closed_form_error_free(k):
    L = 150
    rs = readsim.simulate(6000, L, 10.0, 0.0, k, 7 + k, keep_genome=True)
    genome = rs.genome.tobytes().decode()
    assert len({genome[p:p + k - 1] for p in range(len(genome) - k + 2)}) == len(genome) - k + 2
    assert wide_dict(*oracle.build_graph_wide(rs.reads, rs.offsets, k), k) == closed_form(genome, rs.starts, L, k)


def test_k64_uses_all_126_bits():
    read = "G" * 70 + "T" * 70
    hi, lo, counts = build([read], 64)
    full = [(int(h) << 64) | int(l) for h, l in zip(hi, lo)]
    # G = 3 everywhere: the all-G window is 2^126 - 1
    assert max(full) == (1 << 126) - 1 and int(hi.max()) < (1 << 62)
    # T = 2: the all-T window, the last one of the read
    assert (int("10" * 63, 2)) in full
    assert int(counts.sum()) == len(read) - 64 + 1


def test_single_read_spells_back():
    rng = random.Random(11)
    k = 51
    read = "".join(rng.choice("ACGT") for _ in range(400))
    hi, lo, counts = build([read], k)
    g = wide_dict(hi, lo, counts, k)
    indeg = {v: 0 for v in g}
    for v, out in g.items():
        for c in out:
            indeg[v[1:] + c] += 1
    start = [v for v in g if indeg[v] == 0]
    assert len(start) == 1
    v, s = start[0], start[0]
    while g[v]:
        (c,) = g[v]
        s += c
        v = v[1:] + c
    assert s == read


def test_bounds_and_validation():
    rs = readsim.reads_from_strings(["ACGT" * 20], 40)
    for bad_k in (0, 1, 65, 100):
        with pytest.raises(oracle.OracleError) as e:
            oracle.build_graph_wide(rs.reads, rs.offsets, bad_k)
        assert e.value.code == oracle.E_K
    bad = readsim.reads_from_strings(["ACGT" * 10 + "N" + "ACGT" * 10], 40)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_graph_wide(bad.reads, bad.offsets, 40)
    assert e.value.code == oracle.E_BASE
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_graph_wide(rs.reads, np.array([0, 50, 30, 80], dtype=np.uint64), 40)
    assert e.value.code == oracle.E_INVAL
    hi, lo, counts = build(["A" * 39, ""], 40)
    assert hi.size == 0 and counts.shape == (0, 4)


def test_planted_mistakes_fail_brute_force():
    reads = ["ACGTTGCAAGTC" * 8, "TTGCAAGTCACGT" * 6]
    k = 40
    hi, lo, counts = build(reads, k)
    want = brute.brute_graph(reads, k)
    assert wide_dict(hi, lo, counts, k) == want
    swapped = counts[:, [1, 0, 2, 3]]
    assert wide_dict(hi, lo, swapped, k) != want
    shifted = lo ^ np.uint64(1 << 63)
    assert wide_dict(hi, shifted, counts, k) != want
    assert wide_dict(hi, lo, counts, k + 1) != want
