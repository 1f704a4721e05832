"""GPU: the greedy's launch sequence captured into a HIP graph (HBM_TUNE_SELECT_GRAPH).

Every replay must equal the kernel-by-kernel launches bit for bit: repeated selections on
one store (the kept graph replayed, eager work and synchronisations between replays), a
store that grows (the graph updated in place), a different k (re-instantiated), every
encoding, a full IMM against the oracle, a batch of instances, and the serving loop.
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


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


@pytest.mark.parametrize("enc", ["NONE", "HOT_BITMAP", "HUFFMAN", "HUFFMAN_HOT_BITMAP", "BITMAX"])
def test_graph_replays_equal_eager(P, enc):
    import torch

    g = G.rmat(12, seed=31)
    _say("select graph:", enc, "R-MAT 12 IC-WC")
    ctx = P.Context(0)
    try:
        ctx.load_synth(g, "IC", "WC")
        ctx.hbm_set_encoding(enc, 0.1, 0.01)
        for theta in (5_000, 12_345):  # growing store: same shape, new launch parameters
            ctx.hbm_sample_rr(theta, 42)
            for k in (30, 30, 7, 30):  # replay, replay, a new shape, back again
                ctx.hbm_set_tuning("SELECT_GRAPH", 0)
                ref = ctx.hbm_select_seeds(k)
                ctx.hbm_set_tuning("SELECT_GRAPH", 1)
                for _ in range(3):
                    x = torch.arange(1 << 20, device="cuda").sum().item()  # eager work between replays
                    assert x == (1 << 20) * ((1 << 20) - 1) // 2
                    got = ctx.hbm_select_seeds(k)
                    torch.cuda.synchronize()
                    assert _same(got, ref), (theta, k)
    finally:
        ctx.close()


def test_graph_imm_equals_oracle(orc, P):
    g = G.rmat(13, seed=4)
    q = (40, 0.5, 1.0, 99)
    _say("select graph: IMM R-MAT 13 IC-WC hot bitmap, k 40, against the oracle")
    ctx = P.Context(0)
    try:
        ctx.load_synth(g, "IC", "WC")
        ctx.hbm_set_encoding("HOT_BITMAP", 0.1, 0.01)
        ctx.hbm_set_tuning("SELECT_GRAPH", 1)
        runs = [ctx.hbm_imm(*q) for _ in range(3)]
    finally:
        ctx.close()
    os_, og_, ost, _ = orc.imm(orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC"), *q)
    for seeds, gains, st in runs:
        assert np.array_equal(seeds, os_) and np.array_equal(gains, og_)
        assert st["cov_round"] == ost["cov_round"] and st["theta_round"] == ost["theta_round"]


def test_graph_batch_and_serving(P):
    insts = [(G.rmat(10 + (i % 3), seed=50 + i), "IC" if i % 2 == 0 else "LT") for i in range(6)]
    qs = [(5 + 7 * i, 0.5, 1.0, 300 + i) for i in range(6)]
    _say("select graph: batch of 6 instances, then the serving loop")
    ctxs = []
    try:
        for g, model in insts:
            c = P.Context(0)
            if model == "LT":
                c.hbm_load_graph(g.n, g.row_ptr, g.dst, G.lt_weights(g, 3), model="LT", prob="EDGE")
                c.hbm_set_encoding("HUFFMAN", 0.05, 0.01)
            else:
                c.load_synth(g, "IC", "WC")
                c.hbm_set_encoding("HOT_BITMAP", 0.1, 0.01)
            ctxs.append(c)
        alone = [c.hbm_imm(*q) for c, q in zip(ctxs, qs)]
        ctxs[0].hbm_set_tuning("SELECT_GRAPH", 1)
        for _ in range(2):
            out = P.imm_batch(ctxs, qs)
            for a, b in zip(out, alone):
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        srv = P.Server(ctxs[0], store_budget=1 << 30, max_active=4)
        try:
            sq = [(k, 0.5, 1.0, 700 + i) for i, k in enumerate((10, 25, 5, 40))]
            ref = []
            ctxs[0].hbm_set_tuning("SELECT_GRAPH", 0)
            ref = [ctxs[0].hbm_imm(*q) for q in sq]
            tickets = [srv.hbm_server_submit(*q) for q in sq]
            for t, r in zip(tickets, ref):
                res = srv.hbm_server_poll(t, wait=True)
                assert res["status"] == "OK" and np.array_equal(res["seeds"], r[0]) and np.array_equal(res["gains"], r[1])
        finally:
            srv.close()
    finally:
        for c in ctxs:
            c.close()
