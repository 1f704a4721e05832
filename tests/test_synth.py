"""The synthetic generators (CPU): structure the workloads rely on."""

import numpy as np

from synth import graphs as G


def _check_csr(g):
    rp, d = g.row_ptr, g.dst
    assert rp[0] == 0 and rp[-1] == len(d) and (np.diff(rp) >= 0).all()
    src = g.src()
    assert (src != d).all(), "self-loop"
    key = src.astype(np.int64) * g.n + d
    assert (np.diff(key) > 0).all(), "rows unsorted or duplicate edges"


def test_chung_lu_shape_and_determinism():
    n, avg, top = 20_000, 35.25, 770_155 * 20_000 / 41.7e6
    g = G.chung_lu(n, avg, 2.2, seed=5, max_deg=top)
    _check_csr(g)
    assert abs(g.m / n - avg) / avg < 0.05  # few duplicates at this density
    outd, ind = np.diff(g.row_ptr), g.indeg()
    assert 0.5 * top < outd.max() < 1.5 * top and 0.5 * top < ind.max() < 1.5 * top
    # heavy tail: the top 1% of vertices hold a large share of the edges
    share = np.sort(ind)[::-1][: n // 100].sum() / g.m
    assert share > 0.05  # a uniform graph would give 0.01
    g2 = G.chung_lu(n, avg, 2.2, seed=5, max_deg=top)
    assert np.array_equal(g.row_ptr, g2.row_ptr) and np.array_equal(g.dst, g2.dst)


def test_rmat_and_er_are_clean():
    _check_csr(G.rmat(10, seed=3, cache=False))
    _check_csr(G.erdos_renyi(1024, 8192, seed=1))


def test_serving_queries():
    qs = G.serving_queries(64, seed=5, rate=2.0)
    assert len(qs) == 64 and qs[0]["t"] == 0.0
    t = np.array([q["t"] for q in qs])
    assert (np.diff(t) >= 0).all() and 15 < t[-1] < 50
    assert all(10 <= q["k"] <= 200 and q["eps"] in (0.5, 0.2) for q in qs)
    # a query does not depend on how many are drawn or on the rate, apart from its arrival
    for other in (G.serving_queries(5, seed=5, rate=2.0), G.serving_queries(100, seed=5, rate=0.5)):
        for a, b in zip(qs, other):
            assert (a["k"], a["eps"], a["seed"]) == (b["k"], b["eps"], b["seed"])
    assert [q["t"] * 4 for q in qs[:20]] == [q["t"] for q in G.serving_queries(20, seed=5, rate=0.5)]


def test_batched_instances():
    insts = G.batched_instances()
    assert len(insts) == 256
    assert {i["model"] for i in insts[::2]} == {"IC"} and {i["model"] for i in insts[1::2]} == {"LT"}
    assert all(12 <= i["scale"] <= 18 and 5 <= i["k"] <= 100 and i["eps"] in (0.5, 0.3) for i in insts)


def test_flat_head_graph_is_constant_p():
    g = G.flat_head(2048, 32768, 0.1, seed=2)
    _check_csr(g)
    assert g.m == 32768 and g.w.dtype == np.float32 and (g.w == np.float32(0.1)).all()
    g2 = G.config_graph("flat")
    assert g2.n == 65536 and g2.m == 1 << 20 and (g2.w == np.float32(0.1)).all()
