"""GPU: many IMM instances in shared launches (hbm_imm_batch).

Each instance's result must equal what hbm_imm gives on its context alone, and,
for instances small enough, the oracle's IMM (seeds, gains, theta schedule, LB,
coverage), bit for bit.  The mix follows the batched workload's recipe: R-MAT
graphs of uneven scale, IC weighted cascade with a hot bitmap on even
instances, LT with Huffman on odd ones, k and eps per instance.
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


def _contexts(P, insts):
    ctxs, graphs = [], []
    for inst in insts:
        g = G.instance_graph(inst)
        c = P.Context(0)
        c.load_synth(g, inst["model"], inst["prob"])
        c.hbm_set_encoding(inst["enc"], inst["warmup"], inst["hot"] or 0.01)
        ctxs.append(c)
        graphs.append(g)
    return ctxs, graphs


def _small_mix(count, smin, smax, seed):
    insts = G.batched_instances(count=count, seed=seed, smin=smin, smax=smax)
    for i, inst in enumerate(insts):
        inst["k"] = 5 + (inst["k"] % 30)
    return insts


@pytest.mark.parametrize("block,small", [(1 << 21, 0), (1024, 0), (1 << 21, 1)])
def test_batch_equals_alone_and_oracle(orc, P, block, small):
    insts = _small_mix(10, 8, 11, seed=11)
    _say("batch of", len(insts), "scales", [i["scale"] for i in insts], "block", block, "small tier", small)
    ctxs, graphs = _contexts(P, insts)
    try:
        ctxs[0].hbm_set_tuning("BLOCK_SETS", block)
        ctxs[0].hbm_set_tuning("LDS_SMALL", small)  # the driving context's shape serves the batch
        out = P.imm_batch(ctxs, [(i["k"], i["eps"], i["l"], i["seed"]) for i in insts])
        for inst, c, g, (seeds, gains, st) in zip(insts, ctxs, graphs, out):
            _say("instance", inst["index"], inst["model"], "scale", inst["scale"], "k", inst["k"], "eps", inst["eps"])
            s1, g1, st1 = c.hbm_imm(inst["k"], inst["eps"], inst["l"], inst["seed"])
            assert np.array_equal(seeds, s1) and np.array_equal(gains, g1)
            assert st["theta_round"] == st1["theta_round"] and st["cov_round"] == st1["cov_round"]
            assert st["lb"] == st1["lb"] and st["nsets_final"] == st1["nsets_final"]
            assert st["store"] == st1["store"]
            og = orc.Graph(g.n, g.row_ptr, g.dst, g.w if inst["prob"] == "EDGE" else None, model=inst["model"],
                           prob=inst["prob"])
            os_, og_, ost, _ = orc.imm(og, inst["k"], inst["eps"], inst["l"], inst["seed"])
            assert st["theta_round"] == ost["theta_round"] and st["cov_round"] == ost["cov_round"]
            assert st["lb"] == ost["lb"] and st["theta_final"] == ost["theta_final"]
            assert np.array_equal(seeds, os_) and np.array_equal(gains, og_) and st["coverage"] == ost["coverage"]
    finally:
        for c in ctxs:
            c.close()


def test_batch_full_shape_subset(orc, P):
    """Eight instances of the batched workload itself (scales up to 18): batch == alone,
    and sampled RR sets of each against the oracle."""
    insts = G.batched_instances()[:8]
    _say("workload subset", [(i["index"], i["scale"], i["model"], i["k"], i["eps"]) for i in insts])
    ctxs, graphs = _contexts(P, insts)
    try:
        out = P.imm_batch(ctxs, [(i["k"], i["eps"], i["l"], i["seed"]) for i in insts])
        rng = np.random.default_rng(5)
        for inst, c, g, (seeds, gains, st) in zip(insts, ctxs, graphs, out):
            _say("instance", inst["index"], "theta", st["nsets_final"])
            # the batched store is still on the context: check sampled sets against the oracle
            og = orc.Graph(g.n, g.row_ptr, g.dst, g.w if inst["prob"] == "EDGE" else None, model=inst["model"],
                           prob=inst["prob"])
            T = st["nsets_final"]
            for j in np.unique(np.concatenate([rng.integers(0, T, 200), [0, T - 1]])):
                assert np.array_equal(c.hbm_get_rr(int(j)), og.sample(inst["seed"], int(j))), f"set {j}"
            s1, g1, st1 = c.hbm_imm(inst["k"], inst["eps"], inst["l"], inst["seed"])
            assert np.array_equal(seeds, s1) and np.array_equal(gains, g1)
            assert st["theta_round"] == st1["theta_round"] and st["nsets_final"] == st1["nsets_final"]
            assert st["coverage"] == st1["coverage"] and st["store"] == st1["store"]
    finally:
        for c in ctxs:
            c.close()


def test_batch_instance_errors_are_isolated(P):
    insts = _small_mix(4, 8, 9, seed=3)
    _say("batch with one bad instance")
    ctxs, _ = _contexts(P, insts)
    try:
        qs = [(i["k"], i["eps"], i["l"], i["seed"]) for i in insts]
        qs[2] = (10 ** 6, 0.5, 1.0, 1)  # k > n
        with pytest.raises(P.HbmError) as e:
            P.imm_batch(ctxs, qs)
        assert e.value.status == P.HBM_EINVAL and "instance 2" in str(e.value)
        # the others finished and match their solo runs
        good = [0, 1, 3]
        out = P.imm_batch([ctxs[i] for i in good], [qs[i] for i in good])
        for i, (seeds, _, _) in zip(good, out):
            s1, _, _ = ctxs[i].hbm_imm(*qs[i])
            assert np.array_equal(seeds, s1)
    finally:
        for c in ctxs:
            c.close()


def test_autotune_picks_valid_shapes_and_keeps_results(P):
    insts = _small_mix(6, 9, 11, seed=8)
    _say("autotune over", len(insts), "instances")
    ctxs, _ = _contexts(P, insts)
    try:
        qs = [(i["k"], i["eps"], i["l"], i["seed"]) for i in insts]
        before = P.imm_batch(ctxs, qs)
        tuning, best_ms = P.imm_autotune(ctxs, qs)
        _say("chosen", tuning, "ms", round(best_ms, 2))
        assert tuning["BLOCK_SETS"] in (1 << 16, 1 << 18, 1 << 21)
        assert tuning["IC_T1_BUDGET"] in (1024, 4096, 16384) and tuning["T2_SLOTS"] in (2, 3, 4)
        assert tuning["LT_PATH"] in (32, 64, 128) and best_ms > 0
        assert tuning["LDS_THREADS"] in (0, 512, 1024) and tuning["LDS_PER_CU"] in (0, 2, 3)
        after = P.imm_batch(ctxs, qs)
        for (s0, g0, _), (s1, g1, _) in zip(before, after):
            assert np.array_equal(s0, s1) and np.array_equal(g0, g1)
    finally:
        for c in ctxs:
            c.close()
