"""GPU parity on the served graph at full size: a Chung-Lu digraph shaped like
twitter7 (41.7M vertices, ~1.44B edges, exponent 2.2, weighted cascade), Huffman
+ density-gated hot bitmap.

* Two IMM queries (k=10, eps=.5 and k=120, eps=.2): the theta schedule and the
  final theta against the closed form, 10^4 random RR sets against the oracle one
  by one, the warm-up counts against the oracle's warm-up sets, and the oracle's
  greedy replayed over the GPU's decoded store.
* Served queries (arriving together and later) equal the same queries alone.
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
def served(P):
    import torch

    c = G.C5
    _say("c5 graph: Chung-Lu n", c["n"], "seed", c["gseed"])
    rp, dst = G.chung_lu_csr(c["n"], c["avg_deg"], c["gamma"], c["gseed"], c["max_deg"], device="cuda")
    torch.cuda.synchronize()
    ctx = P.Context(0)
    ctx.hbm_load_graph(c["n"], rp, dst, None, "IC", "WC")
    rp_h, dst_h = rp.cpu().numpy(), dst.cpu().numpy()
    del rp, dst
    torch.cuda.empty_cache()
    ctx.hbm_set_encoding(c["enc"], c["warmup"], c["hot"])
    ctx.hbm_set_hot_density(c["hot_density"])
    yield ctx, c, rp_h, dst_h
    ctx.close()


@pytest.fixture(scope="module")
def c5_oracle(orc, served):
    _, c, rp_h, dst_h = served
    t0 = time.time()
    og = orc.Graph(c["n"], rp_h, dst_h, None, model="IC", prob="WC")
    _say("oracle in-CSR built", round(time.time() - t0, 1), "s")
    return og


@pytest.mark.parametrize("k,eps,seed", [(10, 0.5, 1000), (120, 0.2, 1007)])
def test_c5_query_parity(orc, P, served, c5_oracle, k, eps, seed):
    ctx, c, _, _ = served
    og = c5_oracle
    _say("c5 IMM k", k, "eps", eps, "seed", seed)
    seeds, gains, st = ctx.hbm_imm(k, eps, 1.0, seed)
    T = st["nsets_final"]
    n = c["n"]
    prm = orc.imm_params(n, k, eps, 1.0)
    assert st["lambda_prime"] == prm["lambda_prime"] and st["lambda_star"] == prm["lambda_star"]
    for i, th in enumerate(st["theta_round"], start=1):
        assert th == int(np.ceil(prm["lambda_prime"] / (n / 2.0 ** i)))
    # the final theta from the GPU's last-round coverage by the closed form (Tang et al.'s LB)
    r = st["rounds"]
    th_r, cov_r = st["theta_round"][r - 1], st["cov_round"][r - 1]
    x = n / 2.0 ** r
    ep = np.sqrt(2.0) * eps
    if n * cov_r / th_r >= (1.0 + ep) * x:
        assert st["lb"] == n * cov_r / (th_r * (1.0 + ep))
    assert st["theta_final"] == int(np.ceil(prm["lambda_star"] / st["lb"]))
    # 10^4 random RR indices regenerated one by one by the oracle
    _say("c5 theta", T, "- 10^4 sampled sets against the oracle")
    rng = np.random.default_rng(11 + seed)
    for j in np.unique(np.concatenate([rng.integers(0, T, 10_000), [0, T - 1]])):
        assert np.array_equal(ctx.hbm_get_rr(int(j)), og.sample(seed, int(j))), f"set {j}"
    W = orc.warmup_count(c["warmup"], st["theta_round"][0])
    warm = orc.sample_store(og, seed, W).counts(n)
    assert np.array_equal(ctx.hbm_export("WARM").astype(np.uint64), warm)
    # the oracle's greedy replayed over the GPU's decoded canonical store
    off, mem = ctx.hbm_dump_sets(0, T)
    _say("c5 store dumped:", T, "sets,", int(off[-1]), "members; oracle greedy replay")
    os_, og_, oc = orc.greedy_sets(off, mem, n, k)
    del off, mem
    assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and st["coverage"] == oc


def test_c5_served_equals_alone(P, served):
    ctx, c, _, _ = served
    qs = [(10, 0.5, 1.0, 1000), (40, 0.5, 1.0, 1001), (25, 0.5, 1.0, 1002), (15, 0.5, 1.0, 1003),
          (60, 0.5, 1.0, 1004)]
    alone = {}
    for q in qs:
        alone[q] = ctx.hbm_imm(*q)
    _say("c5 serve: 5 queries, two waves")
    ctx.hbm_set_tuning("BLOCK_SETS", 1 << 16)
    srv = P.Server(ctx, store_budget=c["budget"], max_active=16)
    try:
        tickets = {srv.hbm_server_submit(*q): q for q in qs[:3]}
        time.sleep(0.1)
        tickets.update({srv.hbm_server_submit(*q): q for q in qs[3:]})
        for t, q in tickets.items():
            r = srv.hbm_server_poll(t, wait=True)
            assert r["status"] == "OK", r
            s_, g_, st = alone[q]
            assert np.array_equal(r["seeds"], s_) and np.array_equal(r["gains"], g_)
            assert r["stats"]["nsets_final"] == st["nsets_final"] and r["stats"]["coverage"] == st["coverage"]
        stats = srv.hbm_server_get_stats()
        _say("server stats", stats)
        assert stats["completed"] == len(qs) and stats["peak_active"] >= 2
    finally:
        srv.close()
        ctx.hbm_set_tuning("BLOCK_SETS", 1 << 21)
