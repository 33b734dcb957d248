"""Different handles used from several host threads at once.

The C ABI lets each handle be driven by its own thread (one handle is never
shared between threads).  Here six threads run at the same time, each with
its own handles and its own seeded read sets: binned and direct builds from
host buffers, a captured binned build from device buffers, a merged direct
build, batched builds (whose per-device launch state is shared by every
thread), and captured binned builds whose graph comes out of the same call.
Every graph must equal the oracle's bit for bit.
"""

import threading

import numpy as np
import pytest

import oracle
import readsim
import paper_2401_02756_amd as dbg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROUNDS = 3


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def say(msg):
    print("[case] " + msg, flush=True)


def read_set(worker, r, j=0):
    seed = 0xC0C0 + 1000 * worker + 10 * r + j
    k = 21 if (worker + r) % 2 else 31
    return readsim.simulate(genome_len=30_000 + 7_000 * worker + 3_000 * r, read_len=100 + 50 * (r % 2),
                            coverage=12.0, err=0.01, k=k, seed=seed)


def same(got, want):
    return (got[0].shape == want[0].shape and np.array_equal(got[0], want[0])
            and np.array_equal(got[1], want[1]))


def host_build(flags):
    def run(rs):
        with dbg.Graph(flags=flags) as g:
            g.build(rs.reads, rs.offsets, rs.k)
            return [g.extract_sorted()]
    return run


def device_build(flags):
    def run(rs):
        d_reads = torch.from_numpy(rs.reads).cuda()
        d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
        with dbg.Graph(flags=flags) as g:
            g.build_device(d_reads, d_off, rs.k)
            g.sync()
            return [g.extract_sorted()]
    return run


def fused_build(rs):
    d_reads = torch.from_numpy(rs.reads).cuda()
    d_off = torch.from_numpy(rs.offsets.astype(np.int64)).cuda()
    cap = 400_000
    keys = torch.empty(cap, dtype=torch.int64, device="cuda")
    counts = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    with dbg.Graph(flags=dbg.F_BINNED | dbg.F_GRAPH) as g:
        n = g.build_extract_device(d_reads, d_off, rs.k, keys, counts)
    k = keys.cpu().numpy().view(np.uint64)[:n]
    c = counts.cpu().numpy().view(np.uint32)[:n]
    order = np.argsort(k, kind="stable")
    return [(k[order], c[order])]


def batch_build(sets):
    graphs = [dbg.Graph(flags=dbg.F_BINNED) for _ in sets]
    try:
        st = dbg.build_batch(graphs, [(rs.reads, rs.offsets, rs.k) for rs in sets])
        assert st == [0] * len(sets), st
        return [g.extract_sorted() for g in graphs]
    finally:
        for g in graphs:
            g.close()


WORKERS = [
    ("binned, host input", host_build(dbg.F_BINNED), 1),
    ("direct, host input", host_build(0), 1),
    ("binned, captured, device input", device_build(dbg.F_BINNED | dbg.F_GRAPH), 1),
    ("direct with wave merge, device input", device_build(dbg.F_MERGE), 1),
    ("batched, three graphs", batch_build, 3),
    ("binned build with the vertices written by its reduce", fused_build, 1),
]


def test_handles_on_concurrent_threads():
    inputs, wants = [], []
    for w, (_, _, n) in enumerate(WORKERS):
        sets = [[read_set(w, r, j) for j in range(n)] for r in range(ROUNDS)]
        inputs.append(sets)
        wants.append([[oracle.build_graph(rs.reads, rs.offsets, rs.k) for rs in s] for s in sets])
    say("%d threads x %d rounds on independent handles" % (len(WORKERS), ROUNDS))
    start = threading.Barrier(len(WORKERS))
    errors = [None] * len(WORKERS)

    def work(w):
        name, run, n = WORKERS[w]
        try:
            start.wait()
            for r in range(ROUNDS):
                got = run(inputs[w][r]) if n > 1 else run(inputs[w][r][0])
                for j, (gv, wv) in enumerate(zip(got, wants[w][r])):
                    assert same(gv, wv), "%s: round %d, set %d differs from the oracle" % (name, r, j)
        except BaseException as e:  # reported by the main thread
            errors[w] = e

    threads = [threading.Thread(target=work, args=(w,)) for w in range(len(WORKERS))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
        assert not t.is_alive(), "a worker thread did not finish"
    for w, e in enumerate(errors):
        if e is not None:
            raise AssertionError("%s: %r" % (WORKERS[w][0], e)) from e
