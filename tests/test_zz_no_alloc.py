"""dbg_build_device_static, the build whose scratch lives in the library's
static device array (no allocation), against dbg_build_device on the same
inputs: bit-exact graphs, in both table modes, on two calls in a row (the
second with a smaller input), plus its host-side refusals."""

import numpy as np
import pytest

import oracle
import readsim
import paper_2401_02756_amd as dbg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = [0, dbg.F_BINNED]
MODE_IDS = ["direct", "binned"]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def say(msg):
    print("[case] " + msg, flush=True)


def on_device(rs):
    return (torch.from_numpy(rs.reads).cuda(), torch.from_numpy(rs.offsets.astype(np.int64)).cuda())


def head(rs, n):
    """The first n reads of a read set."""
    end = int(rs.offsets[n])
    return readsim.ReadSet(reads=rs.reads[:end].copy(), offsets=rs.offsets[:n + 1].copy(), k=rs.k,
                           meta=dict(rs.meta))


def same(a, b, what):
    assert a[0].shape == b[0].shape, "%s: %d vs %d vertices" % (what, a[0].shape[0], b[0].shape[0])
    assert np.array_equal(a[0], b[0]), what + ": keys differ"
    assert np.array_equal(a[1], b[1]), what + ": counts differ"


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_static_build_matches_device_build(mode):
    # direct: 34 MB of reads; binned: 6 MB (its records take 16 bytes a base)
    big = readsim.make_instance(4, 9 if mode == dbg.F_BINNED else 3)
    inputs = [big, head(big, big.n_reads // 3), readsim.make_config(1)]
    ev = max(int(rs.meta.get("expected_vertices", 0)) for rs in inputs) + 100_000
    with dbg.Graph(expected_vertices=ev, load_factor=0.5, flags=mode) as g_ref, \
            dbg.Graph(expected_vertices=ev, load_factor=0.5, flags=mode) as g_st:
        for call, rs in enumerate(inputs):
            say("static build, mode %d, call %d: %d reads, k=%d" % (mode, call, rs.n_reads, rs.k))
            d_reads, d_off = on_device(rs)
            g_ref.reset()
            g_st.reset()
            g_ref.build_device(d_reads, d_off, rs.k)
            g_ref.sync()
            g_st.build_device_static(d_reads, d_off, rs.k)
            want = g_ref.extract_sorted()
            got = g_st.extract_sorted()
            same(got, want, "call %d vs dbg_build_device" % call)
            if rs.n_reads <= 2000:
                same(got, oracle.build_graph(rs.reads, rs.offsets, rs.k), "call %d vs oracle" % call)
            st = g_st.stats()
            assert st["inserts"] == int(np.maximum(rs.lengths() - rs.k + 1, 0).sum())
            assert st["vertices"] == got[0].shape[0]
        # builds accumulate as with dbg_build_device
        rs = inputs[-1]
        d_reads, d_off = on_device(rs)
        g_st.build_device_static(d_reads, d_off, rs.k)
        k2, c2 = g_st.extract_sorted()
        wk, wc = oracle.build_graph(rs.reads, rs.offsets, rs.k)
        assert np.array_equal(k2, wk) and np.array_equal(c2, 2 * wc)


def test_static_build_refusals():
    rs = readsim.make_config(1)
    d_reads, d_off = on_device(rs)
    with dbg.Graph(flags=dbg.F_BINNED) as g:  # no table yet: sizing it would allocate
        with pytest.raises(dbg.DbgError) as e:
            g.build_device_static(d_reads, d_off, rs.k)
        assert e.value.code == dbg.E_INVAL
    with dbg.Graph(expected_vertices=50_000, flags=dbg.F_BINNED) as g:
        with pytest.raises(dbg.DbgError) as e:
            g.build_device_static(d_reads, d_off, 33)
        assert e.value.code == dbg.E_K
        # one 40 MB read: its binned pass needs more than the static array
        big = torch.full((40 << 20,), ord("A"), dtype=torch.uint8, device="cuda")
        off = torch.tensor([0, 40 << 20], dtype=torch.int64, device="cuda")
        with pytest.raises(dbg.DbgError) as e:
            g.build_device_static(big, off, 21)
        assert e.value.code == dbg.E_SCRATCH
        assert g.vertex_count() == 0 and g.stats()["builds"] == 0
        g.build_device_static(d_reads, d_off, rs.k)  # the handle is still usable
        got = g.extract_sorted()
    same(got, oracle.build_graph(rs.reads, rs.offsets, rs.k), "after a refused call")
