"""Pins of the oracle's normalized counters (Methods, "Normalization of graph")."""

import numpy as np

import oracle
import readsim
from conftest import read_golden


def test_hand_derived_values():
    for row in read_golden("normalize_hand_derived.txt"):
        genome, total = int(row[1]), int(row[2])
        arrow, semi = row.index("->"), row.index(";")
        counts = np.array([int(x) for x in row[3:arrow]], dtype=np.uint64)
        want32 = [int(x) for x in row[arrow + 1:semi]]
        want8 = [int(x) for x in row[semi + 1:]]
        o32, o8 = oracle.normalize(counts.astype(np.uint32), genome, total)
        assert o32.tolist() == want32, row
        assert o8.tolist() == want8, row


def genome_with_distinct_windows(rng, n, k):
    while True:
        g = "".join(rng.choice(list("ACGT"), size=n))
        if len({g[i:i + k - 1] for i in range(n - k + 2)}) == n - k + 2:
            return g


def test_unique_kmers_normalize_to_one_and_repeats_to_two():
    """A genome read d times end to end: every k-mer is read d times and the
    expected duplication is d (G - k + 1) / G, so a unique k-mer normalizes
    to round(G / (G - k + 1)) = 1; a k-mer the genome holds twice, to 2."""
    rng = np.random.default_rng(4)
    k, d = 21, 7
    unit = genome_with_distinct_windows(rng, 60, k)
    left = genome_with_distinct_windows(rng, 600, k)
    mid = genome_with_distinct_windows(rng, 500, k)
    right = genome_with_distinct_windows(rng, 600, k)
    genome = left + unit + mid + unit + right
    rs = readsim.reads_from_strings([genome] * d, k)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, k)
    total = int(counts.sum())
    assert total == d * (len(genome) - k + 1)
    o32, _ = oracle.normalize(counts, len(genome), total)
    # k-mers inside the repeated unit occur twice in the genome
    inside = {unit[i:i + k] for i in range(len(unit) - k + 1)}
    occurrences = {}
    for i in range(len(genome) - k + 1):
        occurrences[genome[i:i + k]] = occurrences.get(genome[i:i + k], 0) + 1
    letters = "ACTG"
    for key, c, n in zip(keys, counts, o32):
        v = oracle.decode_key(int(key), k)
        for x in range(4):
            if c[x]:
                kmer = v + letters[x]
                assert n[x] == occurrences[kmer], (kmer, c[x], n[x])
    assert any(occurrences[m] == 2 for m in inside)
