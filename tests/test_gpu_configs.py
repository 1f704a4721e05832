"""GPU parity at the benchmark configurations' full sizes, in bench.py's launch configuration.

* R-MAT scale 20, IC weighted cascade, eps=0.5, k=50, hot bitmap (1% of vertices,
  10% warm-up): the oracle runs the whole IMM too, so every round's theta and
  coverage, LB, the seeds, gains and coverage are compared exactly, and the
  encoded store is compared word by word.
* R-MAT scale 23, LT, eps=0.13, k=100, Huffman (5% warm-up): the oracle recomputes
  a random sample of RR sets one by one, and its own greedy is replayed over the
  GPU's decoded store; the codebook, warm-up counts and theta schedule are
  compared exactly.
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


def test_c2_full_imm_parity(orc, P):
    c = G.CONFIGS["c2"]
    _say("c2 full IMM: R-MAT 20 IC-WC eps .5 k 50 hot bitmap, seed 42")
    g = G.config_graph("c2")
    ctx = P.Context(0)
    try:
        ctx.load_synth(g, "IC", "WC")
        ctx.hbm_set_encoding(c["enc"], c["warmup"], c["hot"])
        seeds, gains, st = ctx.hbm_imm(c["k"], c["eps"], c["l"], c["seed"])
        og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
        os_, og_, ost, store = orc.imm(og, c["k"], c["eps"], c["l"], c["seed"])
        assert st["theta_round"] == ost["theta_round"]
        assert st["cov_round"] == ost["cov_round"]
        assert st["lb"] == ost["lb"] and st["theta_final"] == ost["theta_final"]
        assert st["nsets_final"] == ost["nsets_final"]
        assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and st["coverage"] == ost["coverage"]
        # the encoded store, word by word
        W = orc.warmup_count(c["warmup"], ost["theta_round"][0])
        e = orc.Encoded(store, g.n, c["enc"], W, hot_frac=c["hot"])
        assert np.array_equal(ctx.hbm_export("HOT"), e.hot)
        assert np.array_equal(ctx.hbm_export("BITMAP"), e.bitmap)
        assert np.array_equal(ctx.hbm_export("RAW_OFF"), e.cold_off)
        assert np.array_equal(ctx.hbm_export("RAW_MEM"), e.cold_mem)
        assert np.array_equal(ctx.hbm_export("COUNTS").astype(np.uint64), store.counts(g.n))
    finally:
        ctx.close()


def test_c3_sampled_parity_and_greedy_replay(orc, P):
    c = G.CONFIGS["c3"]
    _say("c3: R-MAT 23 LT eps .13 k 100 Huffman, seed 42")
    g = G.config_graph("c3")
    ctx = P.Context(0)
    try:
        ctx.load_synth(g, "LT", "EDGE")
        ctx.hbm_set_encoding(c["enc"], c["warmup"], c["hot"])
        seeds, gains, st = ctx.hbm_imm(c["k"], c["eps"], c["l"], c["seed"])
        T = st["nsets_final"]
        prm = orc.imm_params(g.n, c["k"], c["eps"], c["l"])
        assert st["lambda_prime"] == prm["lambda_prime"] and st["lambda_star"] == prm["lambda_star"]
        for i, th in enumerate(st["theta_round"], start=1):
            assert th == int(np.ceil(prm["lambda_prime"] / (g.n / 2.0 ** i)))
        og = orc.Graph(g.n, g.row_ptr, g.dst, g.w, model="LT", prob="EDGE")
        # sampled sets, one by one
        rng = np.random.default_rng(7)
        idx = np.unique(np.concatenate([rng.integers(0, T, 3000), [0, T - 1]]))
        for j in idx:
            assert np.array_equal(ctx.hbm_get_rr(int(j)), og.sample(c["seed"], int(j))), f"set {j}"
        # warm-up counts and codebook from the oracle's warm-up sets
        W = orc.warmup_count(c["warmup"], st["theta_round"][0])
        ws = orc.sample_store(og, c["seed"], W)
        warm = ws.counts(g.n)
        assert np.array_equal(ctx.hbm_export("WARM").astype(np.uint64), warm)
        assert np.array_equal(ctx.hbm_export("LENS"), orc.huffman_lengths(warm))
        # the oracle's greedy over the GPU's decoded store reproduces the GPU's selection
        off, mem = ctx.hbm_dump_sets(0, T)
        os_, og_, oc = orc.greedy_sets(off, mem, g.n, c["k"])
        assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and st["coverage"] == oc
        assert np.array_equal(ctx.hbm_export("COUNTS").astype(np.uint64),
                              np.bincount(mem, minlength=g.n).astype(np.uint64))
    finally:
        ctx.close()
