"""Randomised parity: small read sets of every kind against the oracle.

Hypothesis draws read sets (short and empty reads, runs of one letter, mixed
case, repeats) and k from 2 to 64; each is built in the direct and the binned
mode, with one or two build calls, and compared with the oracle exactly.  The
draws are derandomised, so every run checks the same cases.
"""

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
import readsim
import paper_2401_02756_amd as dbg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def oracle_records(rs, k):
    if k <= 32:
        return oracle.build_graph(rs.reads, rs.offsets, k)
    hi, lo, counts = oracle.build_graph_wide(rs.reads, rs.offsets, k)
    return np.stack([hi, lo], axis=1), counts


read_text = st.one_of(
    st.text(alphabet="ACGT", min_size=0, max_size=160),
    st.text(alphabet="acgtACGT", min_size=0, max_size=80),
    st.text(alphabet="AC", min_size=0, max_size=120),
    st.builds(lambda c, n: c * n, st.sampled_from("ACGT"), st.integers(0, 150)),
)


@settings(max_examples=200, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(reads=st.lists(read_text, min_size=1, max_size=40), k=st.integers(2, 64),
       binned=st.booleans(), split=st.booleans())
def test_random_read_sets(reads, k, binned, split):
    rs = readsim.reads_from_strings(reads, k)
    want_k, want_c = oracle_records(rs, k)
    flags = dbg.F_BINNED if binned else 0
    with dbg.Graph(flags=flags, expected_vertices=max(64, int(rs.offsets[-1]))) as g:
        if split and len(reads) > 1:
            h = len(reads) // 2
            a = readsim.reads_from_strings(reads[:h], k)
            b = readsim.reads_from_strings(reads[h:], k)
            g.build(a.reads, a.offsets, k)
            g.build(b.reads, b.offsets, k)
        else:
            g.build(rs.reads, rs.offsets, k)
        keys, counts = g.extract_sorted()
    assert keys.shape == want_k.shape
    assert np.array_equal(keys, want_k)
    assert np.array_equal(counts, want_c)
