"""GPU: the serving loop (hbm_server_*).

Queries of different k and eps arrive while others run; each answer must be the
one hbm_imm gives alone on the same graph (seeds, gains, coverage, theta
schedule), bit for bit, whatever the mix, the admission order or preemptions;
two served answers are also checked against the oracle's own IMM.
"""

import sys
import time

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


@pytest.fixture(scope="module")
def graph_ctx(P):
    g = G.rmat(14, seed=21)
    c = P.Context(0)
    c.load_synth(g, "IC", "WC")
    c.hbm_set_encoding("HUFFMAN_HOT_BITMAP", 0.1, 0.001)
    yield c, g
    c.close()


QUERIES = [(10, 0.5, 1.0, 1000), (40, 0.3, 1.0, 1001), (25, 0.5, 1.0, 1002), (60, 0.4, 1.0, 1003),
           (5, 0.5, 1.0, 1004), (80, 0.5, 1.0, 1005)]


@pytest.fixture(scope="module")
def alone(graph_ctx):
    c, _ = graph_ctx
    out = {}
    for q in QUERIES:
        s, g, st = c.hbm_imm(*q)
        out[q] = (s, g, st)
    return out


def _same(res, ref):
    s, g, st = ref
    assert res["status"] == "OK", res
    assert np.array_equal(res["seeds"], s) and np.array_equal(res["gains"], g)
    assert res["stats"]["coverage"] == st["coverage"]
    assert res["stats"]["theta_round"] == st["theta_round"] and res["stats"]["nsets_final"] == st["nsets_final"]
    assert res["stats"]["store"]["store_bytes"] == st["store"]["store_bytes"]


def test_mix_equals_alone(orc, P, graph_ctx, alone):
    c, _ = graph_ctx
    _say("serve: staggered arrivals, budget 4 GB, 4 slots")
    srv = P.Server(c, store_budget=4 << 30, max_active=4)
    try:
        tickets = {}
        for i, q in enumerate(QUERIES):
            tickets[srv.hbm_server_submit(*q)] = q
            if i % 2 == 1:
                time.sleep(0.02)  # later arrivals join running ones
        served = {}
        for t, q in tickets.items():
            r = srv.hbm_server_poll(t, wait=True)
            _say("query", q, "latency ms", round(r["t_done_ms"] - r["t_submit_ms"], 2))
            _same(r, alone[q])
            served[q] = r
        st = srv.hbm_server_get_stats()
        assert st["completed"] == len(QUERIES) and st["failed"] == 0 and st["active"] == 0
        assert st["peak_active"] >= 2  # queries did overlap
    finally:
        srv.close()
    # served answers straight against the oracle's full IMM on the same graph
    g = graph_ctx[1]
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    for q in (QUERIES[1], QUERIES[5]):
        _say("oracle IMM for served query", q)
        os_, og_, ost, _ = orc.imm(og, *q)
        r = served[q]
        assert np.array_equal(r["seeds"], os_) and np.array_equal(r["gains"], og_)
        assert r["stats"]["coverage"] == ost["coverage"] and r["stats"]["theta_round"] == ost["theta_round"]
        assert r["stats"]["lb"] == ost["lb"] and r["stats"]["nsets_final"] == ost["nsets_final"]


def test_budget_preemption_keeps_results(P, graph_ctx, alone):
    """A budget that holds about one store at a time: queries wait or are preempted and
    recomputed, and still return the solo answer."""
    c, _ = graph_ctx
    biggest = max(alone[q][2]["store"]["store_bytes"] for q in QUERIES)
    budget = int(biggest * 1.3)
    _say("serve: tight budget", budget)
    srv = P.Server(c, store_budget=budget, max_active=6)
    try:
        tickets = {srv.hbm_server_submit(*q): q for q in QUERIES}
        for t, q in tickets.items():
            _same(srv.hbm_server_poll(t, wait=True), alone[q])
        st = srv.hbm_server_get_stats()
        _say("stats", st)
        assert st["completed"] == len(QUERIES) and st["peak_store_bytes"] <= budget
    finally:
        srv.close()


def test_bad_and_oversized_queries_fail_alone(P, graph_ctx, alone):
    c, g = graph_ctx
    _say("serve: invalid and oversized queries")
    small = min(alone[q][2]["store"]["store_bytes"] for q in QUERIES)
    srv = P.Server(c, store_budget=max(small // 50, 4096), max_active=2)
    try:
        bad = srv.hbm_server_submit(0, 0.5, 1.0, 1)          # k < 1
        big = srv.hbm_server_submit(80, 0.2, 1.0, 2)         # cannot fit the budget
        rb = srv.hbm_server_poll(bad, wait=True)
        rg = srv.hbm_server_poll(big, wait=True)
        assert rb["status"] == "EINVAL" and rg["status"] == "EBUDGET"
        with pytest.raises(P.HbmError):
            srv.hbm_server_poll(bad)  # forgotten once reported
    finally:
        srv.close()
