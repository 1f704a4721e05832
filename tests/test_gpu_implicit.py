"""GPU parity of implicit roots (hbm_set_implicit_roots): the store leaves each set's root out
of its plain ids or Huffman string and regenerates it from (seed, j).

Every exported array equals the oracle's implicit-root encoding word for word, every set
decodes to the oracle's, selection (plain scan, Huffman partial decode with the root check,
long-string decrement, hot rows) gives the oracle's seeds, a full IMM and a served query
equal the oracle's, and the store is smaller than with explicit roots.
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


CASES = [(enc, model) for enc in ("NONE", "HUFFMAN", "HOT_BITMAP", "HUFFMAN_HOT_BITMAP", "BITMAX")
         for model in ("IC", "LT")]


@pytest.mark.parametrize("enc,model", CASES)
def test_implicit_roots_store_and_selection(orc, P, enc, model):
    g = G.rmat(12, seed=41)
    w = G.lt_weights(g, 2) if model == "LT" else None
    prob = "EDGE" if model == "LT" else "WC"
    theta, seed, frac = 20_000, 77, 0.05
    W = orc.warmup_count(frac, theta)
    _say("implicit roots:", enc, model, "theta", theta)
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
    st = orc.sample_store(og, seed, theta)
    e = orc.Encoded(st, g.n, enc, W=W, hot_frac=0.01, implicit_roots=True)
    ex = orc.Encoded(st, g.n, enc, W=W, hot_frac=0.01)
    out = {}
    for implicit in (True, False):
        ctx = P.Context(0)
        try:
            ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
            ctx.hbm_set_encoding(enc, frac, 0.01)
            ctx.hbm_set_implicit_roots(implicit)
            ctx.hbm_set_tuning("BLOCK_SETS", 6000)  # several blocks: j0 > 0 in the encoders
            ctx.hbm_sample_rr(theta, seed)
            ss = ctx.hbm_get_store_stats()
            if implicit:
                if enc in ("NONE", "HOT_BITMAP"):
                    assert np.array_equal(ctx.hbm_export("RAW_OFF"), e.cold_off)
                    assert np.array_equal(ctx.hbm_export("RAW_MEM"), e.cold_mem)
                if enc in ("HUFFMAN", "HUFFMAN_HOT_BITMAP"):
                    assert np.array_equal(ctx.hbm_export("BITOFF"), e.bitoff)
                    pay = ctx.hbm_export("PAYLOAD")
                    assert np.array_equal(pay, e.payload[:len(pay)])
                if e.nhot:
                    assert np.array_equal(ctx.hbm_export("BITMAP"), e.bitmap)
                off, mem = ctx.hbm_dump_sets(0, theta)
                ooff, omem = st.arrays()
                assert np.array_equal(off, ooff) and np.array_equal(mem, omem)
                assert int(ctx.hbm_get_rr(theta - 1)[0]) == int(omem[ooff[theta - 1]])
            out[implicit] = (ctx.hbm_select_seeds(40), ss)
        finally:
            ctx.close()
    sg, gg, cg = orc.greedy(st, g.n, 40)
    for implicit in (True, False):
        (seeds, gains, cov), _ = out[implicit]
        assert np.array_equal(seeds, sg) and np.array_equal(gains, gg) and cov == cg
    si, se = out[True][1], out[False][1]
    if enc == "BITMAX":
        assert si["store_bytes"] == se["store_bytes"]
    else:
        assert si["store_bytes"] < se["store_bytes"]
        if enc in ("NONE", "HOT_BITMAP"):
            assert se["raw_bytes"] - si["raw_bytes"] == 4 * (ex.cold_off[-1] - e.cold_off[-1])
        else:
            assert se["payload_bits"] - si["payload_bits"] == ex.payload_bits - e.payload_bits


def test_implicit_roots_imm_serving_and_spill(orc, P):
    g = G.rmat(13, seed=17)
    q = (30, 0.5, 1.0, 5)
    _say("implicit roots: IMM (HUFFMAN_HOT_BITMAP), served query, spilled plain store")
    ref = orc.imm(orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC"), *q)
    ctx = P.Context(0)
    try:
        ctx.load_synth(g, "IC", "WC")
        ctx.hbm_set_encoding("HUFFMAN_HOT_BITMAP", 0.05, 0.01)
        ctx.hbm_set_implicit_roots(True)
        seeds, gains, st = ctx.hbm_imm(*q)
        assert np.array_equal(seeds, ref[0]) and np.array_equal(gains, ref[1])
        assert st["cov_round"] == ref[2]["cov_round"] and st["nsets_final"] == ref[2]["nsets_final"]
        srv = P.Server(ctx, store_budget=1 << 30, max_active=4)
        try:
            t = srv.hbm_server_submit(*q)
            r = srv.hbm_server_poll(t, wait=True)
            assert r["status"] == "OK" and np.array_equal(r["seeds"], ref[0])
        finally:
            srv.close()
        ctx.hbm_set_encoding("NONE")
        ctx.hbm_set_implicit_roots(True)
        ctx.hbm_set_spill(4096)
        seeds, gains, st = ctx.hbm_imm(*q)
        assert np.array_equal(seeds, ref[0]) and np.array_equal(gains, ref[1])
    finally:
        ctx.close()
