"""The CPU baseline of the paper's threaded lock-free build
(oracle/lfdbg_cpu.cpp) builds exactly the oracle's graph, for any thread
count and table size -- including a single bucket, where every insertion
races on one list head."""

import numpy as np
import pytest

import oracle
import readsim


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("buckets", [1, 97, 0])
def test_same_graph_as_oracle(threads, buckets):
    if buckets:  # few lists, long chains: a small input
        c1 = readsim.make_config(1)
        n = 150 if buckets == 1 else c1.n_reads
        rs = readsim.reads_from_strings([c1.read(i) for i in range(n)], c1.k)
    else:
        rs = readsim.make_config(2, scale=0.01)
    keys, counts = oracle.build_graph(rs.reads, rs.offsets, rs.k)
    lk, lc, _ = oracle.lfdbg_build(rs.reads, rs.offsets, rs.k, threads, buckets)
    assert np.array_equal(lk, keys) and np.array_equal(lc, counts)


def test_worked_example(worked_example):
    read, k, verts = worked_example
    rs = readsim.reads_from_strings([read], k)
    lk, lc, _ = oracle.lfdbg_build(rs.reads, rs.offsets, k, 2)
    got = {oracle.decode_key(int(x), k): (int(x), c.tolist()) for x, c in zip(lk, lc)}
    assert got == verts


def test_rejects_bad_bytes():
    rs = readsim.reads_from_strings(["ACGTNACGT"], 3)
    with pytest.raises(oracle.OracleError):
        oracle.lfdbg_build(rs.reads, rs.offsets, 3, 2)
