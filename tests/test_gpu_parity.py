"""GPU parity: the HIP library against the CPU oracle, element by element.

Integer results (RR sets, counts, codes, bit streams, seeds, gains, coverage)
must be bit-exact.  Every case prints its name, sizes and seed before it runs.
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


@pytest.fixture()
def ctx(P):
    c = P.Context(0)
    yield c
    c.close()


def _ograph(orc, g, model, prob):
    return orc.Graph(g.n, g.row_ptr, g.dst, g.w if prob == "EDGE" else None, model=model, prob=prob)


def _check_sets(ctx, st, theta, chunk=200_000):
    ooff, omem = st.arrays()
    for j0 in range(0, theta, chunk):
        j1 = min(theta, j0 + chunk)
        off, mem = ctx.hbm_dump_sets(j0, j1)
        ro = ooff[j0:j1 + 1] - ooff[j0]
        assert np.array_equal(off, ro), f"set sizes differ in [{j0},{j1})"
        assert np.array_equal(mem, omem[ooff[j0]:ooff[j1]]), f"set members differ in [{j0},{j1})"


# ---------------------------------------------------------------- graph ingest
@pytest.mark.parametrize("model,prob", [("IC", "EDGE"), ("IC", "WC"), ("LT", "EDGE"), ("LT", "WC")])
def test_transpose_and_thresholds(orc, ctx, model, prob):
    _say("transpose", model, prob)
    g = G.rmat(12, seed=7)
    w = G.lt_weights(g, 8) if model == "LT" else np.random.default_rng(3).random(g.m, dtype=np.float32)
    g = G.with_weights(g, w)
    ctx.load_synth(g, model=model, prob=prob)
    og = _ograph(orc, g, model, prob)
    ptr, src = og.in_csr()
    assert np.array_equal(ctx.hbm_export("IN_PTR"), ptr)
    assert np.array_equal(ctx.hbm_export("IN_SRC"), src)
    thr = ctx.hbm_export("THRESH")
    indeg = np.diff(ptr)
    two24 = np.float32(16777216.0)
    if model == "IC" and prob == "WC":
        p = np.where(indeg > 0, np.float32(1.0) / np.maximum(indeg, 1).astype(np.float32), np.float32(0))
        want = np.ceil(p.astype(np.float32) * two24).astype(np.uint32)
    else:
        # weights in in-edge order
        order = np.lexsort((g.src(), g.dst))
        w_in = g.w[order]
        if prob == "WC":
            w_in = (np.float32(1.0) / np.repeat(indeg, indeg).astype(np.float32)).astype(np.float32)
        if model == "IC":
            want = np.ceil(w_in * two24).astype(np.uint32)
        else:
            want = np.zeros(g.m, dtype=np.uint32)
            for v in range(g.n):
                acc = np.float32(0)
                for e in range(ptr[v], ptr[v + 1]):
                    acc = np.float32(acc + w_in[e])
                    want[e] = np.uint32(np.ceil(np.float32(acc * two24)))
    assert np.array_equal(thr, want)


def test_wc_threshold_division_all_degrees(P, ctx):
    """Per-vertex WC thresholds for every in-degree 1..2000 and one hub of 2^16: 1/d rounded to float32."""
    _say("wc thresholds, all degrees")
    K = 2000
    u, v = [], []
    for d in range(1, K + 1):
        u.extend(range(K + 1, K + 1 + d))
        v.extend([d] * d)
    D = 1 << 16
    u.extend(range(1, D + 1))
    v.extend([0] * D)
    n = max(D, 2 * K) + 1
    g = G._csr_from_pairs(n, np.array(u), np.array(v))
    ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    thr = ctx.hbm_export("THRESH")
    deg = g.indeg()
    p = np.where(deg > 0, np.float32(1.0) / np.maximum(deg, 1).astype(np.float32), np.float32(0.0))
    want = np.ceil(p.astype(np.float32) * np.float32(16777216.0)).astype(np.uint32)
    assert np.array_equal(thr, want)


@pytest.mark.parametrize("bad", ["self_loop", "duplicate", "range", "nan", "negative", "lt_sum", "ic_above_1",
                                 "rowptr"])
def test_invalid_graph_rejected(P, ctx, bad):
    _say("invalid graph", bad)
    n = 6
    rp = np.array([0, 2, 3, 4, 5, 6, 6], dtype=np.int64)
    dst = np.array([1, 2, 3, 4, 5, 0], dtype=np.int32)
    w = np.full(6, 0.5, dtype=np.float32)
    model = "IC"
    if bad == "self_loop":
        dst[0] = 0
    elif bad == "duplicate":
        dst[1] = 1
    elif bad == "range":
        dst[2] = 9
    elif bad == "nan":
        w[3] = np.nan
    elif bad == "negative":
        w[3] = -0.1
    elif bad == "ic_above_1":
        w[3] = 1.5
    elif bad == "lt_sum":
        model = "LT"
        dst[1] = 3  # vertex 3 gets in-edges from 0 and 2
        rp = np.array([0, 2, 3, 4, 5, 6, 6], dtype=np.int64)
        w[:] = 0.75
    elif bad == "rowptr":
        rp[3] = 1
    with pytest.raises(P.HbmError) as ei:
        ctx.hbm_load_graph(n, rp, dst, w, model=model, prob="EDGE")
    assert ei.value.status == P.HBM_EINVAL
    # the context stays usable
    ctx.hbm_load_graph(n, np.array([0, 1, 2, 3, 4, 5, 6], dtype=np.int64), np.array([1, 2, 3, 4, 5, 0], np.int32),
                       np.full(6, 0.5, np.float32), model="IC", prob="EDGE")


def test_state_errors(P, ctx):
    _say("state errors")
    with pytest.raises(P.HbmError) as ei:
        ctx.hbm_sample_rr(10, 1)
    assert ei.value.status == P.HBM_ESTATE
    g = G.erdos_renyi(64, 256, seed=2)
    ctx.load_synth(g, "IC", "EDGE")
    with pytest.raises(P.HbmError) as ei:
        ctx.hbm_select_seeds(0)
    assert ei.value.status == P.HBM_EINVAL
    with pytest.raises(P.HbmError) as ei:
        ctx.hbm_select_seeds(65)
    assert ei.value.status == P.HBM_EINVAL
    with pytest.raises(P.HbmError):
        ctx.hbm_sample_rr(-1, 1)
    with pytest.raises(P.HbmError):
        ctx.hbm_set_encoding("HOT_BITMAP", 0.1, 0.0)


# ---------------------------------------------------------------- RR sets and seeds
def test_c1_tiny_ic_full(orc, ctx):
    """Config C1: ER n=1024 m=8192, p~U[0,0.1], theta=10^4, seed 42, k=10, no compression."""
    _say("c1 full parity")
    g = G.config_graph("c1")
    ctx.load_synth(g, "IC", "EDGE")
    ctx.hbm_set_encoding("NONE")
    ctx.hbm_sample_rr(10_000, 42)
    og = _ograph(orc, g, "IC", "EDGE")
    st = orc.sample_store(og, 42, 10_000)
    _check_sets(ctx, st, 10_000)
    assert np.array_equal(ctx.hbm_export("COUNTS").astype(np.uint64), st.counts(g.n))
    seeds, gains, cov = ctx.hbm_select_seeds(10)
    os_, og_, oc = orc.greedy(st, g.n, 10)
    assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and cov == oc


@pytest.mark.parametrize("model,prob,scale,theta", [("IC", "WC", 14, 30_000), ("LT", "EDGE", 14, 30_000),
                                                    ("IC", "EDGE", 11, 3_000), ("IC", "EDGE", 13, 1_500),
                                                    ("IC", "EDGE", 15, 300), ("IC", "EDGE", 16, 200)])
def test_sets_and_seeds_rmat(orc, ctx, model, prob, scale, theta):
    """Exact RR sets and seeds; with a constant p = 0.25 most sets reach thousands of
    vertices, so the workgroup tiers run: the LDS one and, past its 2048 members, the
    device-bitmap one (at scales 15 and 16 sets of 8-27 K members: sorted runs merged over two and three
    passes)."""
    _say("rmat sets", model, prob, scale, theta)
    g = G.rmat(scale, seed=scale)
    if model == "LT":
        g = G.with_weights(g, G.lt_weights(g, 5))
    elif prob == "EDGE":
        # large RR sets: constant p well above the critical value drives the big-set tier
        g = G.with_weights(g, np.full(g.m, 0.25, dtype=np.float32))
    ctx.load_synth(g, model, prob)
    ctx.hbm_set_encoding("NONE")
    ctx.hbm_sample_rr(theta, 42)
    og = _ograph(orc, g, model, prob)
    st = orc.sample_store(og, 42, theta)
    _check_sets(ctx, st, theta)
    seeds, gains, cov = ctx.hbm_select_seeds(20)
    os_, og_, oc = orc.greedy(st, g.n, 20)
    assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and cov == oc


@pytest.mark.parametrize("queue,lw", [(1 << 20, 32), (300, 32), (1 << 20, 64), (1 << 20, 256)])
def test_lt_long_walks_all_tiers(orc, ctx, queue, lw):
    """A directed path with weight 1: walk length = root id + 1, crossing every LT tier at
    each lane path length (with a 300-entry big-set queue, walks beyond it go through the
    huge-set pass)."""
    _say("lt long walks, big-set queue", queue, "lane path", lw)
    n = 5000
    g = G._csr_from_pairs(n, np.arange(n - 1), np.arange(1, n))
    g = G.with_weights(g, np.ones(g.m, dtype=np.float32))
    ctx.load_synth(g, "LT", "EDGE")
    ctx.hbm_set_tuning("T2_QUEUE", queue)
    ctx.hbm_set_tuning("LT_PATH", lw)
    ctx.hbm_set_encoding("NONE")
    ctx.hbm_sample_rr(400, 9)
    og = _ograph(orc, g, "LT", "EDGE")
    st = orc.sample_store(og, 9, 400)
    _check_sets(ctx, st, 400)


def test_append_equals_direct(orc, ctx):
    _say("append vs direct")
    g = G.rmat(12, seed=3)
    ctx.load_synth(g, "IC", "WC")
    ctx.hbm_set_encoding("NONE")
    ctx.hbm_sample_rr(1000, 5)
    ctx.hbm_sample_rr(2500, 5)
    ctx.hbm_sample_rr(7000, 5)
    og = _ograph(orc, g, "IC", "WC")
    st = orc.sample_store(og, 5, 7000)
    _check_sets(ctx, st, 7000)
    # a new seed resets
    ctx.hbm_sample_rr(500, 6)
    st6 = orc.sample_store(og, 6, 500)
    _check_sets(ctx, st6, 500)


# ---------------------------------------------------------------- encodings
@pytest.mark.parametrize("enc,dens", [("HUFFMAN", 0.0), ("HOT_BITMAP", 0.0), ("HUFFMAN_HOT_BITMAP", 0.0),
                                      ("HUFFMAN_HOT_BITMAP", 1.0 / 32)])
@pytest.mark.parametrize("model", ["IC", "LT"])
def test_encoding_bit_exact(orc, ctx, enc, dens, model):
    _say("encoding", enc, "density gate", dens, model)
    g = G.rmat(13, seed=21)
    prob = "WC" if model == "IC" else "EDGE"
    if model == "LT":
        g = G.with_weights(g, G.lt_weights(g, 4))
    theta, wf, hf = 12_000, 0.1, 0.01
    ctx.load_synth(g, model, prob)
    ctx.hbm_set_encoding(enc, wf, hf)
    ctx.hbm_set_hot_density(dens)
    ctx.hbm_sample_rr(theta, 42)
    og = _ograph(orc, g, model, prob)
    st = orc.sample_store(og, 42, theta)
    W = orc.warmup_count(wf, theta)
    e = orc.Encoded(st, g.n, enc, W, hot_frac=hf, hot_min_density=dens)
    assert np.array_equal(ctx.hbm_export("WARM").astype(np.uint64), e.warm)
    if e.nhot:
        assert np.array_equal(ctx.hbm_export("HOT"), e.hot)
        assert np.array_equal(ctx.hbm_export("BITMAP"), e.bitmap)
    if e.cold_off is not None:
        assert np.array_equal(ctx.hbm_export("RAW_OFF"), e.cold_off)
        assert np.array_equal(ctx.hbm_export("RAW_MEM"), e.cold_mem)
    if e.lens is not None:
        assert np.array_equal(ctx.hbm_export("LENS"), e.lens)
        assert np.array_equal(ctx.hbm_export("CODES"), e.codes)
        assert np.array_equal(ctx.hbm_export("BITOFF"), e.bitoff)
        pay = ctx.hbm_export("PAYLOAD")
        nw = (e.payload_bits + 31) // 32
        assert np.array_equal(pay[:nw], e.payload[:nw])
    stats = ctx.hbm_get_store_stats()
    assert stats["nsets"] == theta and stats["warmup_sets"] == W
    if e.lens is not None:
        assert stats["payload_bits"] == e.payload_bits and stats["escapes"] == e.n_escapes
    _check_sets(ctx, st, theta)
    seeds, gains, cov = ctx.hbm_select_seeds(25)
    os_, og_, oc = orc.greedy(st, g.n, 25)
    assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and cov == oc


# ---------------------------------------------------------------- IMM
@pytest.mark.parametrize("model,enc", [("IC", "HOT_BITMAP"), ("LT", "HUFFMAN"), ("IC", "NONE")])
def test_imm_small(orc, ctx, model, enc):
    _say("imm", model, enc)
    g = G.rmat(13, seed=31)
    prob = "WC" if model == "IC" else "EDGE"
    if model == "LT":
        g = G.with_weights(g, G.lt_weights(g, 6))
    k, eps = 10, 0.5
    ctx.load_synth(g, model, prob)
    ctx.hbm_set_encoding(enc, 0.1, 0.01)
    seeds, gains, st = ctx.hbm_imm(k, eps, 1.0, 42)
    og = _ograph(orc, g, model, prob)
    os_, og_, ost, _ = orc.imm(og, k, eps, 1.0, 42)
    assert st["theta_round"] == ost["theta_round"]
    assert st["cov_round"] == ost["cov_round"]
    assert st["lb"] == ost["lb"] and st["theta_final"] == ost["theta_final"]
    assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and st["coverage"] == ost["coverage"]


@pytest.mark.parametrize("scale,theta,slots,small", [(13, 1_500, 4096, 0), (13, 1_500, 3, 0), (13, 1_500, 0, 0),
                                                    (13, 1_500, 4096, 1), (13, 1_500, 3, 1), (13, 1_500, 0, 1),
                                                    (15, 300, 4096, 1), (15, 300, 2, 0)])
def test_spilled_levels_resume(orc, P, ctx, scale, theta, slots, small):
    """IC sets that outgrow an LDS tier (constant p = 0.25: most sets hold thousands of
    vertices) go on in the next one from the levels it spilled: from the 1024-member tier
    (LDS_SMALL = 1) to the 2048-member one, from there to the extra-large pass, and from that
    pass, past 8192 members, to the device-bitmap tier; or they start over from their root
    when no spill slot is left (few slots: most of them; 0: all).  The sets are the oracle's
    either way."""
    _say("spilled levels resume: scale", scale, "slots", slots, "small tier", small)
    for bad in (-1, 4097):
        assert P.lib().hbm_set_tuning(ctx.h, P.TUNE["SPILL_SLOTS"], bad) == P.HBM_EINVAL
    for bad in (-1, 3):
        assert P.lib().hbm_set_tuning(ctx.h, P.TUNE["LDS_SMALL"], bad) == P.HBM_EINVAL
    g = G.rmat(scale, seed=scale)
    g = G.with_weights(g, np.full(g.m, 0.25, dtype=np.float32))
    ctx.load_synth(g, "IC", "EDGE")
    ctx.hbm_set_encoding("NONE")
    ctx.hbm_set_tuning("SPILL_SLOTS", slots)
    ctx.hbm_set_tuning("LDS_SMALL", small)
    ctx.hbm_sample_rr(theta, 42)
    og = _ograph(orc, g, "IC", "EDGE")
    st = orc.sample_store(og, 42, theta)
    off, _ = st.arrays()
    sizes = np.diff(off)
    if scale == 13:
        assert ((sizes > 2048) & (sizes <= 8192)).sum() > 100  # the extra-large pass ends them
    else:
        assert (sizes > 8192).sum() > 50  # they pass through it to the device-bitmap tier
    _check_sets(ctx, st, theta)


# ---------------------------------------------------------------- launch-shape invariance
@pytest.mark.parametrize("tier1,budget,block,queue,lds", [(0, 0, 1 << 21, 1 << 20, (512, 3)),
                                                          (1, 0, 1 << 21, 1 << 20, (512, 3)),
                                                          (1, 256, 1024, 1 << 20, (1024, 1)),
                                                          (1, 4096, 3000, 1 << 20, (512, 1)),
                                                          (1, 64, 1 << 21, 64, (1024, 2)),
                                                          (1, 128, 1 << 21, 1 << 20, (512, 4)),
                                                          (0, 0, 5000, 100, (1024, 4)),
                                                          (1, 64, 3000, 1 << 20, (512, 3, 1)),
                                                          (0, 0, 1 << 21, 100, (1024, 2, 1))])
def test_tuning_invariance(orc, ctx, tier1, budget, block, queue, lds):
    """Tier choice, tier-1 work budget, block size, big-set queue size (small queues
    send sets to the huge-set pass) and the LDS tier's workgroup shape change speed
    only, never the sets."""
    _say("tuning invariance", tier1, budget, block, queue, lds)
    g = G.rmat(14, seed=14)
    ctx.load_synth(g, "IC", "WC")
    ctx.hbm_set_tuning("IC_TIER1", tier1)
    ctx.hbm_set_tuning("IC_T1_BUDGET", budget)
    ctx.hbm_set_tuning("BLOCK_SETS", block)
    ctx.hbm_set_tuning("T2_QUEUE", queue)
    ctx.hbm_set_tuning("LDS_THREADS", lds[0])
    ctx.hbm_set_tuning("LDS_PER_CU", lds[1])
    ctx.hbm_set_tuning("LDS_SMALL", lds[2] if len(lds) > 2 else 0)  # the 1024-member tier in front
    ctx.hbm_set_encoding("HOT_BITMAP", 0.1, 0.01)
    theta = 20_000
    ctx.hbm_sample_rr(theta, 42)
    og = _ograph(orc, g, "IC", "WC")
    st = orc.sample_store(og, 42, theta)
    _check_sets(ctx, st, theta)
    seeds, gains, cov = ctx.hbm_select_seeds(15)
    os_, og_, oc = orc.greedy(st, g.n, 15)
    assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and cov == oc


@pytest.mark.parametrize("enc", ["NONE", "HUFFMAN"])
def test_argmax_coverage_complete_before_k(orc, ctx, enc):
    """The store is covered long before the k-th pick: the remaining picks are the lowest
    unselected ids (count 0), with dense counts and with sparse slots, whose scan for that id
    looks only at ids below k."""
    n, theta, k = 3001, 40, 150
    _say("argmax: coverage complete before k", enc)
    g = G.erdos_renyi(n, 6000, seed=5)
    ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
    ctx.hbm_set_encoding(enc, 0.5, 0.02)
    ctx.hbm_sample_rr(theta, 3)
    og = _ograph(orc, g, "IC", "EDGE")
    st = orc.sample_store(og, 3, theta)
    os_, og_, oc = orc.greedy(st, g.n, k)
    assert oc == theta and og_[-1] == 0  # every set covered, the last picks gain nothing
    for sparse in (0, 1):
        ctx.hbm_set_tuning("SPARSE_COUNTS", sparse)
        seeds, gains, cov = ctx.hbm_select_seeds(k)
        assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and cov == oc, f"SPARSE_COUNTS={sparse}"


# ---------------------------------------------------------------- argmax edge cases
@pytest.mark.parametrize("n,m,enc,k", [(1000, 6000, "NONE", 1000), (5003, 40000, "HUFFMAN", 5003),
                                       (9001, 90000, "HOT_BITMAP", 200), (9001, 90000, "HUFFMAN_HOT_BITMAP", 64)])
def test_argmax_ragged_and_exhaustive(orc, ctx, n, m, enc, k):
    """Greedy seeds equal the oracle's, ties to the lowest id included, where n leaves a
    count tail past the last 4-vertex group (5003, 9001) and where k = n selects every
    vertex, down to those of count 0; with dense counts and with sparse slots (vertices
    outside the store win only as the lowest unselected id)."""
    _say("argmax edge cases", n, m, enc, k)
    g = G.erdos_renyi(n, m, seed=n)
    ctx.hbm_load_graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
    ctx.hbm_set_encoding(enc, 0.1, 0.02)
    theta = 20_000
    ctx.hbm_sample_rr(theta, 7)
    og = _ograph(orc, g, "IC", "EDGE")
    st = orc.sample_store(og, 7, theta)
    os_, og_, oc = orc.greedy(st, g.n, k)
    for sparse in (0, 1):
        ctx.hbm_set_tuning("SPARSE_COUNTS", sparse)
        seeds, gains, cov = ctx.hbm_select_seeds(k)
        assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and cov == oc, f"SPARSE_COUNTS={sparse}"
