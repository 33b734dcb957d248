"""Pins of the oracle's contigs (Methods, "Finding contigs", Algorithm 5).

The oracle's contig walk is checked against hand-derived cases, closed forms
of error-free reads, and an independent checker: every contig must be a walk
of the graph that starts on an out-edge of a start vertex, passes only
one-edge vertices it has not passed before, and stops exactly where the rule
says; every out-edge of every start vertex begins exactly one contig.  That
pins the whole contig set, which is unique under the rule.
"""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import readsim
from conftest import read_golden
from oracle import brute


def golden_cases():
    cases, cur = [], None
    for row in read_golden("contigs_hand_derived.txt"):
        if row[0] == "case":
            cur = (row[1], int(row[2]), row[3:], [])
            cases.append(cur)
        else:
            cur[3].append(row[1].encode())
    return cases


def contigs_of(reads, k):
    rs = readsim.reads_from_strings(reads, k)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, k)
    return oracle.contig_strings(*oracle.contigs(keys, counts, k))


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: c[0])
def test_hand_derived_contigs(case):
    name, k, reads, want = case
    assert contigs_of(reads, k) == sorted(want)


def test_error_free_read_is_one_contig():
    rng = np.random.default_rng(5)
    for k in (5, 11, 21, 31, 32):
        for _ in range(20):
            while True:  # distinct (k-1)-mers, so the read's graph is a simple path
                s = "".join(rng.choice(list("ACGT"), size=int(rng.integers(k, 300))))
                if len({s[i:i + k - 1] for i in range(len(s) - k + 2)}) == len(s) - k + 2:
                    break
            assert contigs_of([s], k) == [s.encode()]


def test_tiling_reads_of_a_genome_give_the_genome():
    rng = np.random.default_rng(9)
    k = 21
    for _ in range(10):
        while True:
            g = "".join(rng.choice(list("ACGT"), size=2000))
            if len({g[i:i + k - 1] for i in range(len(g) - k + 2)}) == len(g) - k + 2:
                break
        # reads of 150 bases every 100 bases (overlaps of 50 >= k - 1), shuffled
        reads = [g[i:i + 150] for i in range(0, len(g) - 150 + 1, 100)] + [g[-150:]]
        rng.shuffle(reads)
        assert contigs_of(reads, k) == [g.encode()]


def graph_dict(reads, k):
    """Graph from the brute-force enumeration: {vertex: [count per letter A C T G]}."""
    return {v: [e.get(a, 0) for a in "ACTG"] for v, e in brute.brute_graph(list(reads), k).items()}


def check_contig_set(contigs, g, k):
    """The checker: each contig follows the rule; each start edge begins one."""
    letters = "ACTG"
    out = {v: [letters[c] for c in range(4) if cnt[c]] for v, cnt in g.items()}
    has_in = {v: False for v in g}
    for v, ls in out.items():
        for a in ls:
            has_in[v[1:] + a] = True
    starts = {v for v in g if out[v] and (len(out[v]) >= 2 or not has_in[v])}
    begun = []
    for s in contigs:
        s = s.decode()
        assert len(s) >= k, s
        vs = [s[i:i + k - 1] for i in range(len(s) - k + 2)]
        assert vs[0] in starts, s
        for i in range(len(vs) - 1):
            assert s[i + k - 1] in out[vs[i]], s  # every step is an edge
        for i in range(1, len(vs) - 1):  # passed vertices: one edge, first visit
            assert len(out[vs[i]]) == 1 and vs[i] not in vs[:i], s
        last = vs[-1]
        assert len(out[last]) != 1 or last in vs[:-1], s  # stops exactly where the rule says
        begun.append((vs[0], s[k - 1]))
    assert sorted(begun) == sorted((v, a) for v in starts for a in out[v])


@settings(max_examples=150, deadline=None)
@given(st.data())
def test_contigs_pass_the_independent_checker(data):
    k = data.draw(st.integers(2, 7))
    alphabet = data.draw(st.sampled_from(["AC", "ACG", "ACGT"]))
    reads = data.draw(st.lists(st.text(alphabet, min_size=0, max_size=40), min_size=1, max_size=12))
    check_contig_set(contigs_of(reads, k), graph_dict(reads, k), k)


def test_checker_catches_planted_mistakes():
    reads = ["ACGTTGCAACGTAGCATGCA", "TTGCAACG", "GCATGCAAT"]
    k = 4
    g = graph_dict(reads, k)
    good = contigs_of(reads, k)
    check_contig_set(good, g, k)
    longest = max(good, key=len)
    mutants = [
        [c for c in good if c != good[0]],                                  # a contig dropped
        [c[:-1] if c == longest else c for c in good],                       # stopped one edge early
        good + [good[0]],                                                    # a contig twice
    ]
    # walked one edge past a vertex with several out-edges
    letters = "ACTG"
    for c in good:
        last = c[-(k - 1):].decode()
        outs = [letters[i] for i in range(4) if g[last][i]]
        if len(outs) >= 2:
            mutants.append([x + outs[0].encode() if x == c else x for x in good])
            break
    for bad in mutants:
        with pytest.raises(AssertionError):
            check_contig_set(bad, g, k)


def test_digest_is_order_free_and_sensitive():
    d = oracle.strings_digest(np.frombuffer(b"ACGTTTTACGGA", dtype=np.uint8),
                              np.array([0, 4, 7, 12], dtype=np.uint64))  # ACGT, TTT, ACGGA
    same = oracle.strings_digest(np.frombuffer(b"ACGGAACGTTTT", dtype=np.uint8),
                                 np.array([0, 5, 9, 12], dtype=np.uint64))  # ACGGA, ACGT, TTT
    other = oracle.strings_digest(np.frombuffer(b"ACGGAACGTTTA", dtype=np.uint8),
                                  np.array([0, 5, 9, 12], dtype=np.uint64))
    split = oracle.strings_digest(np.frombuffer(b"ACGGAACGTTTT", dtype=np.uint8),
                                  np.array([0, 5, 8, 12], dtype=np.uint64))
    assert d == same and d != other and d != split
