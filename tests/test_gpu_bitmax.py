"""GPU parity of the all-vertex Bitmax store and Alg. 1's automatic choice.

* BITMAX (the Bitmax encoding section): the n-row bit matrix word for word against the
  oracle's, every decoded set, and the greedy seeds against both the oracle's plain greedy
  and its Alg. 3 run on the bit matrix; IC and LT; theta not a multiple of 64.
* AUTO (Alg. 1): a flat-head store (constant-p IC on a graph where most roots reach a giant
  in-component: Eq. 2 skewness < 0, density > 1/32) is coded as Bitmax, a skewed one
  (weighted cascade on R-MAT) as Huffmax, both as the oracle decides; a full IMM under AUTO
  equals the oracle's IMM and its store is smaller than plain ids.
"""

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


def _flat(n=4096, m=65536, p=0.1, seed=3):
    g = G.erdos_renyi(n, m, seed=seed)
    g.w = np.full(g.m, p, dtype=np.float32)
    return g


@pytest.mark.parametrize("model", ["IC", "LT"])
def test_bitmax_store_and_selection(orc, P, model):
    if model == "IC":
        g = _flat()
        w = g.w
    else:
        g = G.rmat(10, seed=8)
        w = G.lt_weights(g, 4)
    theta, W, seed = 3001, 150, 42
    _say("bitmax", model, "n", g.n, "m", g.m, "theta", theta)
    ctx = P.Context(0)
    try:
        ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, w, model=model, prob="EDGE")
        ctx.hbm_set_encoding("BITMAX", W / theta, 0.01)
        ctx.hbm_sample_rr(theta, seed)
        og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob="EDGE")
        st = orc.sample_store(og, seed, theta)
        e = orc.Encoded(st, g.n, "BITMAX", W=orc.warmup_count(W / theta, theta))
        ss = ctx.hbm_get_store_stats()
        assert ss["encoding"] == 4 and ss["nhot"] == g.n and ss["raw_bytes"] == 0 and ss["index_bytes"] == 0
        assert ss["store_bytes"] == ss["bitmap_bytes"] == e.nwords * g.n * 8
        assert np.array_equal(ctx.hbm_export("HOT"), e.hot)
        assert np.array_equal(ctx.hbm_export("BITMAP"), e.bitmap)
        ooff, omem = st.arrays()
        off, mem = ctx.hbm_dump_sets(0, theta)
        assert np.array_equal(off, ooff) and np.array_equal(mem, omem)
        for k in (1, 25, 200):
            seeds, gains, cov = ctx.hbm_select_seeds(k)
            s3, g3, c3 = e.bitmax_select(k)
            sg, gg, cg = orc.greedy(st, g.n, k)
            assert np.array_equal(seeds, s3) and np.array_equal(gains, g3) and cov == c3
            assert np.array_equal(seeds, sg) and cov == cg
    finally:
        ctx.close()


def test_auto_choice_matches_oracle(orc, P):
    cases = [("flat-head ER, IC p=.1", _flat(), "IC", "EDGE", "BITMAX"),
             ("R-MAT 12, IC weighted cascade", G.rmat(12, seed=21), "IC", "WC", "HUFFMAN")]
    for name, g, model, prob, want in cases:
        theta, seed = 2000, 7
        _say("auto:", name)
        ctx = P.Context(0)
        try:
            w = g.w if prob == "EDGE" else None
            ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
            ctx.hbm_set_encoding("AUTO", 0.1, 0.01)
            ctx.hbm_sample_rr(theta, seed)
            og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
            st = orc.sample_store(og, seed, theta)
            W = orc.warmup_count(0.1, theta)
            e = orc.Encoded(st, g.n, "AUTO", W=W)
            ss = ctx.hbm_get_store_stats()
            S, D = st.characterize(g.n, 0, W)
            assert e.enc_name == want and ss["encoding"] == orc.ENC[want], (S, D)
            assert ss["skewness"] == S and ss["density"] == D
            if want == "BITMAX":
                assert np.array_equal(ctx.hbm_export("BITMAP"), e.bitmap)
            else:
                assert np.array_equal(ctx.hbm_export("PAYLOAD"), e.payload[:len(ctx.hbm_export("PAYLOAD"))])
                assert np.array_equal(ctx.hbm_export("BITOFF"), e.bitoff)
            seeds, gains, cov = ctx.hbm_select_seeds(30)
            sg, gg, cg = orc.greedy(st, g.n, 30)
            assert np.array_equal(seeds, sg) and np.array_equal(gains, gg) and cov == cg
        finally:
            ctx.close()


def test_auto_imm_flat_head(orc, P):
    g = _flat(16384, 262144, 0.1, seed=5)
    k, eps, l, seed = 20, 0.5, 1.0, 42
    _say("auto IMM: ER 16384/262144 IC p=.1 k", k, "eps", eps)
    ctx = P.Context(0)
    try:
        ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
        ctx.hbm_set_encoding("AUTO", 0.1, 0.01)
        seeds, gains, st = ctx.hbm_imm(k, eps, l, seed)
        og = orc.Graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
        os_, og_, ost, store = orc.imm(og, k, eps, l, seed)
        assert st["theta_round"] == ost["theta_round"] and st["cov_round"] == ost["cov_round"]
        assert st["lb"] == ost["lb"] and st["nsets_final"] == ost["nsets_final"]
        assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and st["coverage"] == ost["coverage"]
        sto = st["store"]
        assert sto["encoding"] == 4  # Bitmax chosen
        raw = 4 * sto["members"] + 8 * (sto["nsets"] + 1)
        _say("B/RR bitmax", sto["store_bytes"] / sto["nsets"], "raw", raw / sto["nsets"])
        assert sto["store_bytes"] < raw
    finally:
        ctx.close()
