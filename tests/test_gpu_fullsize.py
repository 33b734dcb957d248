"""Parity at the full workload sizes, in the launch configurations the
benchmark times: every vertex of every graph against the oracle.

  * bacterial scale (5 Mbp, 120M k-mers): the step's dbg_build_extract_device
    output (load factor 0.4, a replayed captured pass) and dbg_extract of the
    table, each sorted and compared element by element;
  * large (100 Mbp, 1.6G k-mers, 510M vertices): the benchmark's step (binned,
    load factor 0.5, a replayed captured pass) and dbg_extract of the table,
    against the oracle run as 16 key-space partitions in parallel threads
    (each partition of the oracle is exact for its keys);
  * batched (256 read sets, 2.3G k-mers): one batched pass at load factor 0.4
    (the autotuner's usual choice) and one at 0.5, every set;
  * served: all 64 read sets of the served workload's pool submitted to one
    server in a shuffled mix, every request's graph.

Graph records are compared unsorted (tests/records.py): each record is looked
up among the oracle's, counters compared, and every oracle record must be met
exactly once.  The oracle runs as (read set, key-space partition) tasks on 16
host threads, largest first; a task compares its slice as soon as it is
built, so oracle output never accumulates.
"""

import concurrent.futures
import threading

import numpy as np
import pytest

import oracle
import readsim
import records
import paper_2401_02756_amd as dbg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THREADS = 16  # host threads of the oracle
PART_INSERTS = 120_000_000  # a read set above this is split into key-space partitions


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    records.lib()
    yield


def say(msg):
    print("[case] " + msg, flush=True)


def same(got, want, what):
    gk, gc = got
    wk, wc = want
    assert gk.shape == wk.shape, "%s: %d vertices, oracle has %d" % (what, gk.shape[0], wk.shape[0])
    assert np.array_equal(gk, wk), what + ": keys differ"
    bad = int(np.count_nonzero(np.any(gc != wc, axis=1)))
    assert bad == 0, "%s: %d vertices have different counts" % (what, bad)


def kmers(rs):
    return int(np.maximum(rs.lengths() - rs.k + 1, 0).sum())


def parts_for(inserts):
    return max(1, -(-int(inserts) // PART_INSERTS))


class Job:
    """One read set whose graph records (from one or more outputs) are checked
    against the oracle, partition by partition.  got() returns the list of
    (what, keys, counts) outputs; it is called once, on first use."""

    def __init__(self, name, rs, parts, got):
        self.name, self.rs, self.parts, self._got = name, rs, parts, got
        self.lock = threading.Lock()
        self.outputs = None
        self.part_of = None
        self.left = parts

    def fetch(self):
        with self.lock:
            if self.outputs is None:
                self.outputs = self._got()
                if self.parts > 1:
                    self.part_of = [oracle.partition_of(k, self.parts) for _, k, _ in self.outputs]
            return self.outputs, self.part_of

    def done_one(self):
        with self.lock:
            self.left -= 1
            if self.left == 0:
                self.outputs = self.part_of = None


def run_oracle_checks(jobs):
    """Every (job, partition) task on THREADS host threads, costliest first;
    returns the number of vertices checked."""
    tasks = [(j, p) for j in jobs for p in range(j.parts)]
    tasks.sort(key=lambda t: -kmers(t[0].rs) / t[0].parts)
    checked = [0]
    lock = threading.Lock()

    def one(task):
        job, p = task
        rs = job.rs
        want = oracle.build_graph(rs.reads, rs.offsets, rs.k, job.parts, p)
        outputs, part_of = job.fetch()
        for o, (what, keys, counts) in enumerate(outputs):
            records.assert_exact(want, (keys, counts), "%s, %s, partition %d of %d" % (job.name, what, p, job.parts),
                                 part_of[o] if part_of is not None else None, p)
        with lock:
            checked[0] += want[0].shape[0]
        job.done_one()

    with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
        for f in [ex.submit(one, t) for t in tasks]:
            f.result()
    return checked[0]


def test_bacterial_full_exact():
    rs = readsim.make_config(2)
    say("bacterial scale: %d reads, k=%d" % (rs.n_reads, rs.k))
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    with dbg.Graph(expected_vertices=rs.meta["expected_vertices"], load_factor=0.4,
                   flags=dbg.F_BINNED | dbg.F_GRAPH) as g:
        cap = int(g.stats()["capacity"])
        d_keys = torch.empty(cap, dtype=torch.int64, device="cuda")
        d_counts = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
        for _ in range(2):  # the second build replays the captured pass
            g.reset()
            n = g.build_extract_device(d_reads, d_off, rs.k, d_keys, d_counts)
        keys = d_keys[:n].cpu().numpy().view(np.uint64)
        counts = d_counts[:n].cpu().numpy().view(np.uint32)
        order = np.argsort(keys, kind="stable")
        from_table = g.extract_sorted()
    want = oracle.build_graph_parallel(rs.reads, rs.offsets, rs.k, threads=THREADS)
    same((keys[order], counts[order]), want, "bacterial, the step's output")
    same(from_table, want, "bacterial, dbg_extract")


@pytest.mark.timeout(900)
def test_large_full_exact():
    rs = readsim.make_config(3)
    ins = kmers(rs)
    say("large: %d reads, %d bases, k=%d" % (rs.n_reads, rs.total_bases, rs.k))
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    with dbg.Graph(expected_vertices=rs.meta["expected_vertices"], load_factor=0.5,
                   flags=dbg.F_BINNED | dbg.F_GRAPH) as g:
        cap = int(g.stats()["capacity"])
        d_keys = torch.empty(cap, dtype=torch.int64, device="cuda")
        d_counts = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
        for _ in range(2):  # the benchmark's step; the second replays the captured pass
            g.reset()
            n = g.build_extract_device(d_reads, d_off, rs.k, d_keys, d_counts)
        say("large: %d vertices" % n)
        step_keys = d_keys[:n].cpu().numpy().view(np.uint64)
        step_counts = d_counts[:n].cpu().numpy().view(np.uint32)
        del d_keys, d_counts
        torch.cuda.empty_cache()
        st = g.stats()
        table_keys, table_counts = g.extract()
    del d_reads, d_off
    torch.cuda.empty_cache()
    assert st["inserts"] == ins and st["vertices"] == n
    # ~713 buckets of ~713 segments: both scatters take big tiles, the first their 128 KB form
    assert (st["bin_shape1"], st["bin_shape2"]) == (dbg.SHAPE_BIG_WIDE, dbg.SHAPE_BIG), st
    assert int(step_counts.sum(dtype=np.uint64)) == ins
    job = Job("large", rs, 16, lambda: [("the step's output", step_keys, step_counts),
                                        ("dbg_extract", table_keys, table_counts)])
    say("large: oracle in 16 key-space partitions, every vertex compared")
    assert run_oracle_checks([job]) == n


def _batch_layout(sets):
    lens = np.concatenate([x.lengths() for x in sets])
    offs = np.zeros(lens.shape[0] + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    rb = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([x.n_reads for x in sets], out=rb[1:])
    return offs, rb


@pytest.mark.timeout(600)
def test_batched_full_exact():
    n = 256
    with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
        sets = list(ex.map(lambda j: readsim.make_instance(4, j), range(n)))
    offs, rb = _batch_layout(sets)
    ks = [x.k for x in sets]
    say("batched: %d sets, %d reads, load factors 0.4 and 0.5" % (n, int(rb[-1])))
    d_reads = torch.from_numpy(np.concatenate([x.reads for x in sets])).cuda()
    d_off = torch.from_numpy(offs).cuda()
    lfs = (0.4, 0.5)
    graphs = {lf: [dbg.Graph(expected_vertices=readsim.instance_params(4, j)["expected_vertices"], load_factor=lf,
                             flags=dbg.F_BINNED | dbg.F_GRAPH) for j in range(n)] for lf in lfs}
    try:
        for lf in lfs:
            assert dbg.build_batch_device(graphs[lf], rb, ks, d_reads, d_off) == [0] * n
            for j, (g, x) in enumerate(zip(graphs[lf], sets)):
                assert g.stats()["inserts"] == kmers(x), (lf, j)
        del d_reads, d_off

        def outputs(j):
            return lambda: [("load factor %.1f" % lf,) + graphs[lf][j].extract() for lf in lfs]

        jobs = [Job("set %d" % j, x, parts_for(kmers(x)), outputs(j)) for j, x in enumerate(sets)]
        checked = run_oracle_checks(jobs)
        assert checked == sum(g.vertex_count() for g in graphs[0.5])
        say("batched: %d vertices checked, each at both load factors" % checked)
    finally:
        for lf in lfs:
            for g in graphs[lf]:
                g.close()


@pytest.mark.timeout(900)
def test_served_full_exact():
    pool_n = 64
    with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
        sets = list(ex.map(lambda j: readsim.make_instance(5, j), range(pool_n)))
    say("served: all %d pool read sets (%d k-mers) in one shuffled mix" % (pool_n, sum(kmers(x) for x in sets)))
    order = list(np.random.default_rng(0xC5).permutation(pool_n))
    with dbg.Server() as srv:
        ids = {}
        for j in order:
            x = sets[j]
            ids[j] = srv.submit_device(torch.from_numpy(x.reads).cuda(),
                                       torch.from_numpy(x.offsets.astype(np.int64)).cuda(), x.k,
                                       x.meta["expected_vertices"])
        for j in order:
            assert srv.wait(ids[j], timeout=300.0) == dbg.OK, j
        st = srv.stats()
        say("served: %d passes, at most %d in flight" % (st["passes"], st["max_in_flight"]))

        def outputs(j):
            return lambda: [("request %d" % ids[j],) + srv.graph(ids[j]).extract()]

        jobs = [Job("payload %d" % j, x, parts_for(kmers(x)), outputs(j)) for j, x in enumerate(sets)]
        checked = run_oracle_checks(jobs)
        say("served: %d vertices checked" % checked)
        for j in order:
            assert srv.graph(ids[j]).stats()["inserts"] == kmers(sets[j])
            srv.release(ids[j])
