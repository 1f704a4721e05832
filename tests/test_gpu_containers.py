"""GPU parity of the hot set's array rows (hbm_set_row_containers): hot vertices below warm-up
density 1/16 keep, per chunk of 2^16 sets, the ascending 16-bit offsets of their sets.

Over three chunks (the last one ragged) filled by blocks that straddle chunk boundaries, every
exported array equals the oracle's container encoding word for word (array rows, their chunk
offsets and entries, the bitmap rows, the plain ids or Huffman stream), every set decodes to
the oracle's, and selection (u* with an array row, a bitmap row or none; array-row counts
decremented) gives the oracle's seeds.  A full IMM, a batched IMM, a served query and the
selection that allocates nothing give the oracle's answers too, and the store shrinks.
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


CASES = [(enc, model, implicit) for enc in ("HOT_BITMAP", "HUFFMAN_HOT_BITMAP") for model in ("IC", "LT")
         for implicit in (False, True)]


@pytest.mark.parametrize("enc,model,implicit", CASES)
def test_containers_store_and_selection(orc, P, enc, model, implicit):
    g = G.rmat(12, seed=23)
    w = G.lt_weights(g, 3) if model == "LT" else None
    prob = "EDGE" if model == "LT" else "WC"
    theta, seed, frac, hot = 150_000, 91, 0.04, 0.05
    W = orc.warmup_count(frac, theta)
    _say("containers:", enc, model, "implicit", implicit, "theta", theta)
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
    st = orc.sample_store(og, seed, theta)
    e = orc.Encoded(st, g.n, enc, W=W, hot_frac=hot, implicit_roots=implicit, containers=True)
    plain = orc.Encoded(st, g.n, enc, W=W, hot_frac=hot, implicit_roots=implicit)
    assert e.nar > 0 and e.nhot > 0 and e.nchunks == 3
    sizes = {}
    for containers in (True, False):
        ctx = P.Context(0)
        try:
            ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
            ctx.hbm_set_encoding(enc, frac, hot)
            ctx.hbm_set_implicit_roots(implicit)
            ctx.hbm_set_row_containers(containers)
            ctx.hbm_set_tuning("BLOCK_SETS", 40_000)  # blocks straddle the chunk boundaries
            ctx.hbm_sample_rr(theta, seed)
            ss = ctx.hbm_get_store_stats()
            sizes[containers] = ss
            if not containers:
                assert ss["narray"] == 0 and ss["array_bytes"] == 0
                continue
            assert ss["narray"] == e.nar and ss["nhot"] == e.nhot and ss["array_entries"] == len(e.ar_low)
            assert np.array_equal(ctx.hbm_export("ARR_HOT"), e.ar_hot)
            assert np.array_equal(ctx.hbm_export("ARR_OFF"), e.ar_off)
            assert np.array_equal(ctx.hbm_export("ARR_LOW"), e.ar_low)
            assert np.array_equal(ctx.hbm_export("HOT"), e.hot)
            assert np.array_equal(ctx.hbm_export("BITMAP"), e.bitmap)
            if enc == "HOT_BITMAP":
                assert np.array_equal(ctx.hbm_export("RAW_OFF"), e.cold_off)
                assert np.array_equal(ctx.hbm_export("RAW_MEM"), e.cold_mem)
            else:
                assert np.array_equal(ctx.hbm_export("BITOFF"), e.bitoff)
                pay = ctx.hbm_export("PAYLOAD")
                assert np.array_equal(pay, e.payload[:len(pay)])
            off, mem = ctx.hbm_dump_sets(0, theta)
            ooff, omem = st.arrays()
            assert np.array_equal(off, ooff) and np.array_equal(mem, omem)
            for k in (1, 60, 400):
                seeds, gains, cov = ctx.hbm_select_seeds(k)
                sg, gg, cg = orc.greedy(st, g.n, k)
                assert np.array_equal(seeds, sg) and np.array_equal(gains, gg) and cov == cg, k
                # the greedy picks vertices of each kind
                if k == 400:
                    assert set(seeds.tolist()) & set(e.ar_hot.tolist())
                    assert set(seeds.tolist()) & set(e.hot.tolist())
            ns, ng, nc = ctx.hbm_select_seeds_noalloc(60)
            sg, gg, cg = orc.greedy(st, g.n, 60)
            assert np.array_equal(ns, sg) and np.array_equal(ng, gg) and nc == cg
        finally:
            ctx.close()
    # the array rows' bytes, counted in store_bytes, replace bitmap rows worth more
    si, sp = sizes[True], sizes[False]
    assert si["array_bytes"] == e.nchunks * (e.nar + 1) * 8 + 2 * len(e.ar_low)
    assert si["bitmap_bytes"] == 8 * e.nwords * e.nhot and sp["bitmap_bytes"] == 8 * plain.nwords * plain.nhot
    assert si["store_bytes"] < sp["store_bytes"]


def test_containers_imm_batch_and_serving(orc, P):
    g = G.rmat(13, seed=31)
    queries = [(40, 0.5, 1.0, 8), (15, 0.4, 1.0, 9)]
    _say("containers: IMM, batch, served query")
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    refs = [orc.imm(og, *q) for q in queries]
    ctxs = []
    try:
        for enc in ("HOT_BITMAP", "HUFFMAN_HOT_BITMAP"):
            ctx = P.Context(0)
            ctxs.append(ctx)
            ctx.load_synth(g, "IC", "WC")
            ctx.hbm_set_encoding(enc, 0.05, 0.05)
            ctx.hbm_set_row_containers(True)
            for q, ref in zip(queries, refs):
                seeds, gains, st = ctx.hbm_imm(*q)
                assert np.array_equal(seeds, ref[0]) and np.array_equal(gains, ref[1])
                assert st["cov_round"] == ref[2]["cov_round"] and st["nsets_final"] == ref[2]["nsets_final"]
                assert st["store"]["narray"] > 0
        res = P.imm_batch(ctxs, queries)
        for (seeds, gains, st), ref in zip(res, refs):
            assert np.array_equal(seeds, ref[0]) and np.array_equal(gains, ref[1])
        srv = P.Server(ctxs[1], store_budget=1 << 30, max_active=4)
        try:
            t = srv.hbm_server_submit(*queries[0])
            r = srv.hbm_server_poll(t, wait=True)
            assert r["status"] == "OK" and np.array_equal(r["seeds"], refs[0][0])
        finally:
            srv.close()
    finally:
        for c in ctxs:
            c.close()


def test_containers_setting_errors(P):
    ctx = P.Context(0)
    try:
        assert P.lib().hbm_set_row_containers(ctx.h, 2) == P.HBM_EINVAL
        assert P.lib().hbm_set_row_containers(ctx.h, -1) == P.HBM_EINVAL
        assert P.lib().hbm_set_row_containers(ctx.h, 1) == P.HBM_OK
    finally:
        ctx.close()
