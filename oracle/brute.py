"""Brute-force graph of tiny inputs -- TEST INFRASTRUCTURE ONLY.

A second way to the same result as the C core, by sorting instead of hashing
and on strings instead of packed keys, so that a mistake in one is unlikely to
be repeated in the other.  From the definition (Background, the A-Bruijn
graph paragraph): the vertices are the distinct (k-1)-substrings at every
window of every read of length >= k, including the last window, which is only
a target; the edge counter of (vertex, letter) is the number of occurrences of
the k-mer vertex+letter over all reads.
"""

from __future__ import annotations

import itertools


def brute_graph(reads: list[str], k: int) -> dict:
    """{vertex string: {letter: count}} with zero counters omitted."""
    reads = [r.upper() for r in reads]
    windows = sorted(r[j:j + k - 1] for r in reads if len(r) >= k
                     for j in range(len(r) - k + 2))
    vertices = [w for w, _ in itertools.groupby(windows)]
    kmers = sorted(r[j:j + k] for r in reads for j in range(len(r) - k + 1))
    graph = {v: {} for v in vertices}
    for kmer, run in itertools.groupby(kmers):
        graph[kmer[:-1]][kmer[-1]] = sum(1 for _ in run)
    return graph
