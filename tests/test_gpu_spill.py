"""GPU: plain-id stores spilled past a device cap to pinned host memory (hbm_set_spill).

Where the ids live must not change any result: the spilled store decodes to the oracle's
sets, exports the same id array, and selection and a full IMM give the oracle's seeds,
gains and coverage, for caps that put the split inside a set, at a 16-byte boundary, and
past the whole store.
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


@pytest.mark.parametrize("enc,cap", [("NONE", 16), ("NONE", 4000), ("NONE", 1 << 30), ("HOT_BITMAP", 1000)])
def test_spilled_store_parity(orc, P, enc, cap):
    g = G.rmat(12, seed=23)
    theta, seed, k = 20_000, 42, 40
    _say("spill", enc, "cap", cap, "R-MAT 12 IC-WC theta", theta)
    ctx = P.Context(0)
    try:
        ctx.load_synth(g, "IC", "WC")
        ctx.hbm_set_encoding(enc, 0.1, 0.01)
        ctx.hbm_set_spill(cap)
        ctx.hbm_sample_rr(theta // 3, seed)  # grown in several requests: host part copied on growth
        ctx.hbm_sample_rr(theta, seed)
        og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
        st = orc.sample_store(og, seed, theta)
        ooff, omem = st.arrays()
        off, mem = ctx.hbm_dump_sets(0, theta)
        assert np.array_equal(off, ooff) and np.array_equal(mem, omem)
        if enc == "NONE":
            assert np.array_equal(ctx.hbm_export("RAW_MEM"), omem)
        seeds, gains, cov = ctx.hbm_select_seeds(k)
        s2, g2, c2 = orc.greedy(st, g.n, k)
        assert np.array_equal(seeds, s2) and np.array_equal(gains, g2) and cov == c2
    finally:
        ctx.close()


def test_spilled_imm_equals_device_imm(orc, P):
    g = G.rmat(13, seed=9)
    q = (25, 0.5, 1.0, 7)
    _say("spill IMM: R-MAT 13 IC-WC k 25 eps .5, cap 64 KiB vs no cap vs oracle")
    ref = orc.imm(orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC"), *q)
    out = []
    for cap in (0, 1 << 16):
        ctx = P.Context(0)
        try:
            ctx.load_synth(g, "IC", "WC")
            ctx.hbm_set_encoding("NONE")
            ctx.hbm_set_spill(cap)
            out.append(ctx.hbm_imm(*q))
        finally:
            ctx.close()
    for seeds, gains, st in out:
        assert np.array_equal(seeds, ref[0]) and np.array_equal(gains, ref[1])
        assert st["coverage"] == ref[2]["coverage"] and st["nsets_final"] == ref[2]["nsets_final"]


def test_spill_argument_checks(P):
    ctx = P.Context(0)
    try:
        for bad in (-1, 1, 15):
            with pytest.raises(P.HbmError):
                ctx.hbm_set_spill(bad)
        ctx.hbm_set_spill(0)
    finally:
        ctx.close()
