"""The selection entry point that allocates nothing (hbm_select_seeds_noalloc), called
through the C ABI, against hbm_select_seeds on the same stores: two calls in a row, the
second on a smaller input, must each give the same seeds, gains and coverage bit for bit;
a store whose selection state exceeds the fixed scratch is refused with EINVAL."""

import sys

import numpy as np
import pytest

from synth import graphs as G

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2208_00613_amd as P

    P.lib()
    return P


def _store(P, g, model, prob, enc, theta, seed):
    c = P.Context(0)
    c.load_synth(g, model=model, prob=prob)
    c.hbm_set_encoding(enc, 0.05, 0.01)
    c.hbm_sample_rr(theta, seed)
    return c


def test_noalloc_matches_select_two_calls(P):
    _say("noalloc: R-MAT 14 IC-WC Huffman theta=40000 k=60, then R-MAT 11 LT hot bitmap theta=3000 k=17")
    big = _store(P, G.rmat(14, seed=5), "IC", "WC", "HUFFMAN", 40_000, 42)
    gs = G.rmat(11, seed=6)
    gs.w = G.lt_weights(gs, 9)
    small = _store(P, gs, "LT", "EDGE", "HOT_BITMAP", 3_000, 7)
    ref_big = big.hbm_select_seeds(60)
    ref_small = small.hbm_select_seeds(17)
    got_big = big.hbm_select_seeds_noalloc(60)
    got_small = small.hbm_select_seeds_noalloc(17)  # second call in a row, smaller input
    for ref, got in ((ref_big, got_big), (ref_small, got_small)):
        assert np.array_equal(ref[0], got[0]), "seeds differ"
        assert np.array_equal(ref[1], got[1]), "gains differ"
        assert ref[2] == got[2], "coverage differs"
    # and back to the larger store: state left by the smaller call must not leak
    again = big.hbm_select_seeds_noalloc(60)
    assert np.array_equal(again[0], ref_big[0]) and np.array_equal(again[1], ref_big[1])
    big.close()
    small.close()


def test_noalloc_plain_store_and_k_equal_n(P):
    _say("noalloc: ER 1024/8192 IC-EDGE plain theta=10000, k=10 then k=n")
    g = G.erdos_renyi(1024, 8192, seed=1)
    c = _store(P, g, "IC", "EDGE", "NONE", 10_000, 42)
    for k in (10, g.n):
        ref = c.hbm_select_seeds(k)
        got = c.hbm_select_seeds_noalloc(k)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1]) and ref[2] == got[2]
    c.close()


def test_noalloc_refuses_oversized_state(P):
    _say("noalloc: 2^24-vertex path graph, selection state above the scratch -> EINVAL")
    n = 1 << 24
    src = np.arange(0, 4096, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:4097] = np.arange(1, 4097)
    row_ptr[4097:] = 4096
    dst = (src + 1).astype(np.int32)
    c = P.Context(0)
    c.hbm_load_graph(n, row_ptr, dst, None, model="IC", prob="WC")
    c.hbm_set_encoding("NONE")
    c.hbm_sample_rr(1000, 3)
    with pytest.raises(P.HbmError) as e:
        c.hbm_select_seeds_noalloc(5)
    assert e.value.status == P.HBM_EINVAL
    ref = c.hbm_select_seeds(5)  # the allocating call still works on that store
    assert len(ref[0]) == 5
    c.close()
