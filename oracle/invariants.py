"""Properties every correct graph satisfies -- TEST INFRASTRUCTURE ONLY.

These checks hold at any input size, so they also serve where the full oracle
build is too large to run.  They follow from the definition of the graph
(Background, the A-Bruijn graph paragraph) and from the post-condition of the
build loop (both vertices of every k-mer exist once it is added):

  * total:   the counters sum to the number of k-mers, sum over reads of
             max(0, L - k + 1);
  * closure: every edge (v, c) with a non-zero counter leads to a vertex that
             exists, namely (v << 2 | c) masked to 2(k-1) bits;
  * balance: for every vertex, out-degree minus in-degree (edge multiplicities)
             equals the number of reads whose first window is v minus the
             number whose last window is v -- each read is a walk.

``sort_build`` is a third, vectorised way to the graph (numpy sort and
run-length), used to cross-check the C core at sizes the string brute force
cannot reach.
"""

from __future__ import annotations

import numpy as np

# ASCII -> counter index, the paper's (c >> 1) & 3, for the four letters only.
_CODE = np.full(256, 255, dtype=np.uint8)
for _ch in b"ACGTacgt":
    _CODE[_ch] = (_ch >> 1) & 3


def expected_total(offsets, k: int) -> int:
    lens = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(np.maximum(lens - k + 1, 0).sum())


def _codes(reads) -> np.ndarray:
    c = _CODE[np.asarray(reads, dtype=np.uint8)]
    if c.size and c.max() == 255:
        raise ValueError("non-ACGT byte in reads")
    return c.astype(np.uint64)


def _pack_at(codes: np.ndarray, starts: np.ndarray, length: int) -> np.ndarray:
    """Keys of the `length`-mers beginning at each start, first base high."""
    key = np.zeros(starts.shape[0], dtype=np.uint64)
    for i in range(length):
        key = (key << np.uint64(2)) | codes[starts + i]
    return key


def end_windows(reads, offsets, k: int):
    """Keys of the first and of the last window of every read with L >= k."""
    off = np.asarray(offsets, dtype=np.int64)
    lens = np.diff(off)
    ok = lens >= k
    codes = _codes(reads)
    first = _pack_at(codes, off[:-1][ok], k - 1)
    last = _pack_at(codes, off[1:][ok] - (k - 1), k - 1)
    return first, last


def sort_build(reads, offsets, k: int):
    """Graph as (keys ascending, counts[V, 4]) by sorting all windows."""
    off = np.asarray(offsets, dtype=np.int64)
    lens = np.diff(off)
    ok = lens >= k
    codes = _codes(reads)
    nwin = np.where(ok, lens - k + 2, 0)
    read_of = np.repeat(np.arange(lens.shape[0]), nwin)
    first_win = np.cumsum(nwin) - nwin
    j = np.arange(int(nwin.sum()), dtype=np.int64) - np.repeat(first_win, nwin)
    starts = off[:-1][read_of] + j
    keys = _pack_at(codes, starts, k - 1)
    is_edge = j <= (lens[read_of] - k)
    vert = np.unique(keys)
    counts = np.zeros((vert.shape[0], 4), dtype=np.uint32)
    ek = keys[is_edge]
    el = codes[starts[is_edge] + (k - 1)].astype(np.int64)
    idx = np.searchsorted(vert, ek)
    np.add.at(counts, (idx, el), 1)
    return vert, counts


def check_graph(keys, counts, reads, offsets, k: int) -> None:
    """Raise AssertionError naming the first property that fails."""
    keys = np.asarray(keys, dtype=np.uint64)
    counts = np.asarray(counts, dtype=np.uint64).reshape(-1, 4)
    assert keys.shape[0] == counts.shape[0], "keys/counts length mismatch"
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    counts = counts[order]
    V = keys.shape[0]
    if V:
        assert np.all(keys[1:] != keys[:-1]), "duplicate vertex"
    mask = np.uint64((1 << (2 * (k - 1))) - 1)
    assert V == 0 or int(keys[-1]) <= int(mask), "key wider than 2(k-1) bits"

    total = int(counts.sum())
    want = expected_total(offsets, k)
    assert total == want, "total count %d != sum(L-k+1) = %d" % (total, want)

    # closure and in-degree
    u, c = np.nonzero(counts)
    tgt = ((keys[u] << np.uint64(2)) | c.astype(np.uint64)) & mask
    pos = np.searchsorted(keys, tgt)
    pos_c = np.minimum(pos, max(V - 1, 0))
    assert np.all((pos < V) & (keys[pos_c] == tgt)), "edge to a missing vertex"
    indeg = np.zeros(V, dtype=np.int64)
    np.add.at(indeg, pos, counts[u, c].astype(np.int64))
    outdeg = counts.sum(axis=1).astype(np.int64)

    first, last = end_windows(reads, offsets, k)
    bal = np.zeros(V, dtype=np.int64)
    if first.size:
        pf = np.searchsorted(keys, first)
        pl = np.searchsorted(keys, last)
        assert np.all(keys[np.minimum(pf, V - 1)] == first), "first window not a vertex"
        assert np.all(keys[np.minimum(pl, V - 1)] == last), "last window not a vertex"
        np.add.at(bal, pf, 1)
        np.add.at(bal, pl, -1)
    bad = np.nonzero(outdeg - indeg != bal)[0]
    assert bad.size == 0, "degree balance fails at %d vertices (first key %d)" % (
        bad.size, int(keys[bad[0]]) if bad.size else -1)
