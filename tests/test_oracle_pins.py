"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them:

* Philox4x32-10 against the published known-answer vectors;
* the Bitmax worked example of Eq. 3 (bitmap rows, first and second seed);
* RR sets against textbook reverse reachability when every edge is live,
  and against {root} when none is; the root is always a member (Eq. 2's
  remark that every RR set holds its starting vertex);
* exact enumeration of live-edge worlds on graphs with at most 14 edges:
  membership probabilities and the RIS estimator n * F_R(S) (Background, RIS);
* greedy max coverage against brute force marginal gains and the (1 - 1/e)
  bound over all k-subsets (Background, greedy / submodularity);
* IMM's theta against Eq. 1's printed form, and IMM's seeds within
  (1 - 1/e - eps) of the brute-force optimum of exact influence;
* Huffman lengths against the heap-merge optimum and the Kraft equality,
  decode(encode(R)) == R (the coding is lossless: Huffmax encoding section);
* Eq. 2's skewness and density against scipy and the definition.
"""

import itertools
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.stats

from synth import graphs as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox
def test_philox_kat(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_root_uniform(orc):
    n = 37
    roots = np.array([orc.root(n, 42, j) for j in range(37000)])
    assert roots.min() >= 0 and roots.max() < n
    cnt = np.bincount(roots, minlength=n)
    chi2 = ((cnt - 1000.0) ** 2 / 1000.0).sum()
    # 36 degrees of freedom; P(chi2 > 80) ~ 3e-5
    assert chi2 < 80


# ---------------------------------------------------------------- Eq. 3
def _eq3():
    d = {}
    for line in open(os.path.join(GOLD, "eq3_bitmap_example.txt")):
        if line.strip() and line[0] != "#":
            k, *v = line.split()
            d[k] = v
    before = np.array([[int(c) for c in r] for r in d["before"]], dtype=np.int64)
    after = np.array([[int(c) for c in r] for r in d["after"]], dtype=np.int64)
    return before, after, int(d["first_ustar"][0])


def _sets_from_rows(rows):
    nv, ns = rows.shape
    sets = [np.nonzero(rows[:, j])[0].astype(np.int32) for j in range(ns)]
    off = np.zeros(ns + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in sets])
    return off, np.concatenate(sets).astype(np.int32)


def test_eq3_greedy(orc):
    before, after, first = _eq3()
    off, mem = _sets_from_rows(before)
    seeds, gains, cov = orc.greedy_sets(off, mem, n=5, k=2)
    assert seeds[0] == first
    # the rows after subtracting u* hold the remaining counts; the next pick is their argmax
    rest = after.sum(axis=1)
    assert gains[1] == rest.max()
    assert seeds[1] == int(np.argmax(rest))
    assert int(gains[0]) == int(before[first].sum())
    assert cov == 6
    # k = 3: every set is covered, the third pick has gain 0 and is the lowest unselected id
    seeds3, gains3, cov3 = orc.greedy_sets(off, mem, n=5, k=3)
    assert list(seeds3[:2]) == list(seeds) and gains3[2] == 0 and seeds3[2] == 1 and cov3 == 6


def test_eq3_bitmap_rows(orc):
    """Encoding the example's columns as RR sets with every vertex hot must give the printed rows."""
    before, _, _ = _eq3()
    off, mem = _sets_from_rows(before)
    st = _store_from_sets(orc, off, mem, n=5)
    enc = orc.Encoded(st, 5, "HOT_BITMAP", W=6, hot_frac=1.0)
    assert enc.nwords == 1
    rows = {}
    for r, v in enumerate(enc.hot):
        word = int(enc.bitmap[r])
        rows[int(v)] = [(word >> j) & 1 for j in range(6)]
    for v in range(5):
        assert rows[v] == list(before[v])


def test_subtract_identity_exhaustive():
    v = np.arange(256, dtype=np.uint16)[:, None]
    u = np.arange(256, dtype=np.uint16)[None, :]
    assert np.array_equal(v & (v ^ u), v & (~u & 0xFF))


# ---------------------------------------------------------------- helpers
def _store_from_sets(orc, off, mem, n):
    return orc.Store.from_sets(off, mem)


# ---------------------------------------------------------------- RR sets: special cases
def _reverse_reach(n, row_ptr, dst, v):
    A = sp.csr_matrix((np.ones(len(dst)), dst, row_ptr), shape=(n, n))
    order = csg.breadth_first_order(A.T.tocsr(), v, directed=True, return_predecessors=False)
    return np.sort(order)


@pytest.mark.parametrize("prob", ["EDGE", "WC"])
def test_ic_all_live_is_reverse_reach(orc, prob):
    g = G.rmat(9, seed=5)
    w = np.ones(g.m, dtype=np.float32)
    og = orc.Graph(g.n, g.row_ptr, g.dst, w if prob == "EDGE" else None, model="IC", prob=prob)
    if prob == "WC":
        # WC is all-live only for in-degree-1 vertices; use a graph where every in-degree is <= 1
        n = 300
        rng = np.random.default_rng(0)
        parent = np.array([rng.integers(0, v) if v > 0 else -1 for v in range(n)])
        u = parent[1:]
        v = np.arange(1, n)
        tg = G._csr_from_pairs(n, u, v)
        og = orc.Graph(tg.n, tg.row_ptr, tg.dst, None, model="IC", prob="WC")
        g = tg
    for j in range(200):
        s = og.sample(7, j)
        r = orc.root(g.n, 7, j)
        assert np.array_equal(s, _reverse_reach(g.n, g.row_ptr, g.dst, r))


def test_ic_none_live_is_root(orc):
    g = G.rmat(9, seed=5)
    og = orc.Graph(g.n, g.row_ptr, g.dst, np.zeros(g.m, dtype=np.float32), model="IC", prob="EDGE")
    for j in range(300):
        assert list(og.sample(3, j)) == [orc.root(g.n, 3, j)]


def test_lt_chain_and_zero(orc):
    n = 50
    g = G._csr_from_pairs(n, np.arange(n - 1), np.arange(1, n))
    og = orc.Graph(n, g.row_ptr, g.dst, np.ones(g.m, dtype=np.float32), model="LT", prob="EDGE")
    for j in range(100):
        r = orc.root(n, 9, j)
        assert list(og.sample(9, j)) == list(range(r + 1))
    og0 = orc.Graph(n, g.row_ptr, g.dst, np.zeros(g.m, dtype=np.float32), model="LT", prob="EDGE")
    for j in range(100):
        assert list(og0.sample(9, j)) == [orc.root(n, 9, j)]


def test_lt_cycle_stops(orc):
    # a directed 5-cycle with weight 1: the walk visits all 5 vertices and stops at the repeat
    n = 5
    g = G._csr_from_pairs(n, np.arange(n), (np.arange(n) + 1) % n)
    og = orc.Graph(n, g.row_ptr, g.dst, np.ones(n, dtype=np.float32), model="LT", prob="EDGE")
    for j in range(20):
        assert list(og.sample(1, j)) == list(range(n))


@pytest.mark.parametrize("model,prob", [("IC", "EDGE"), ("IC", "WC"), ("LT", "EDGE")])
def test_root_member_and_sorted(orc, model, prob):
    g = G.rmat(10, seed=11)
    w = G.lt_weights(g, 3) if model == "LT" else np.full(g.m, 0.3, dtype=np.float32)
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob=prob)
    for j in range(500):
        s = og.sample(42, j)
        assert orc.root(g.n, 42, j) in set(s.tolist())
        assert np.all(np.diff(s) > 0)


# ---------------------------------------------------------------- exact enumeration
def _tiny(seed, n, m, lt=False):
    g = G.tiny_graph(n, m, seed, p_lo=0.05, p_hi=0.95)
    if lt:
        g = G.with_weights(g, G.lt_weights(g, seed + 1))
    return g


def _effective_ic_p(p):
    # the coin compares a 24-bit draw with p * 2^24 in float32
    return np.ceil(p.astype(np.float64) * 2 ** 24) / 2 ** 24


def _exact_ic_member_prob(g):
    """P[u in RR(v)] for all u, v, by enumerating all 2^m live-edge worlds."""
    n, m = g.n, g.m
    src = g.src()
    p = _effective_ic_p(g.w)
    P = np.zeros((n, n))
    for mask in range(1 << m):
        live = np.array([(mask >> e) & 1 for e in range(m)], dtype=bool)
        pr = np.prod(np.where(live, p, 1 - p))
        A = np.zeros((n, n), dtype=bool)
        A[src[live], g.dst[live]] = True
        # reach[u, v]: u reaches v in the live graph
        R = np.eye(n, dtype=bool)
        for _ in range(n):
            R = R | (R.astype(np.int64) @ A.astype(np.int64) > 0)
        P += pr * R
    return P  # P[u, v] = P[u reaches v] = P[u in RR(v)]


def _exact_lt_member_prob(g):
    """P[u in RR(v)] by enumerating every vertex's choice of at most one in-edge."""
    n = g.n
    src = g.src()
    ins = [[] for _ in range(n)]
    for e in range(g.m):
        ins[g.dst[e]].append(e)
    # effective probabilities of the float32 cumulative thresholds
    choices = []
    for v in range(n):
        es = sorted(ins[v], key=lambda e: src[e])
        acc = np.float32(0)
        prev = 0.0
        opts = []
        for e in es:
            acc = np.float32(acc + g.w[e])
            t = min(math.ceil(float(acc) * 2 ** 24), 2 ** 24) / 2 ** 24
            opts.append((src[e], t - prev))
            prev = t
        opts.append((None, 1.0 - prev))
        choices.append(opts)
    P = np.zeros((n, n))
    for combo in itertools.product(*choices):
        pr = np.prod([c[1] for c in combo])
        if pr == 0:
            continue
        for v in range(n):
            seen = {v}
            cur = v
            while True:
                s = combo[cur][0]
                if s is None or s in seen:
                    break
                seen.add(s)
                cur = s
            for u in seen:
                P[u, v] += pr
    return P


@pytest.mark.parametrize("lt,seed", [(False, 1), (False, 2), (True, 3), (True, 4)])
def test_membership_matches_enumeration(orc, lt, seed):
    g = _tiny(seed, n=6, m=12 if not lt else 11, lt=lt)
    P = _exact_lt_member_prob(g) if lt else _exact_ic_member_prob(g)
    og = orc.Graph(g.n, g.row_ptr, g.dst, g.w, model="LT" if lt else "IC", prob="EDGE")
    theta = 120_000
    st = orc.sample_store(og, 1234 + seed, theta)
    cnt = st.counts(g.n).astype(np.float64)
    pu = P.mean(axis=1)  # root uniform: P[u in RR] = mean_v P[u in RR(v)]
    z = (cnt - theta * pu) / np.sqrt(theta * pu * (1 - pu) + 1e-12)
    assert np.all(np.abs(z) < 5), z
    # RIS: n * F_R(S) estimates E[I(S)] = sum_v P[S reaches v]; check for all pairs S
    off, mem = st.arrays()
    setid = np.repeat(np.arange(theta), np.diff(off))
    for S in itertools.combinations(range(g.n), 2):
        hit = np.zeros(theta, dtype=bool)
        hit[setid[np.isin(mem, S)]] = True
        F = hit.mean()
        # exact P[S hits RR(v)] needs the joint law; bound it with inclusion-exclusion on one world set
        # instead, compare with enumeration of the union directly
        exact = _exact_union_prob(g, S, lt)
        zz = (F - exact) / math.sqrt(exact * (1 - exact) / theta + 1e-15)
        assert abs(zz) < 5, (S, F, exact)


_UNION_CACHE = {}


def _exact_union_prob(g, S, lt):
    """P[S intersects RR(v)] averaged over a uniform root v, by enumeration (cached per graph)."""
    key = (g.name, lt)
    if key not in _UNION_CACHE:
        _UNION_CACHE[key] = _exact_reach_table(g, lt)
    worlds = _UNION_CACHE[key]
    tot = 0.0
    for pr, R in worlds:
        tot += pr * R[list(S), :].any(axis=0).mean()
    return tot


def _exact_reach_table(g, lt):
    n = g.n
    src = g.src()
    out = []
    if not lt:
        p = _effective_ic_p(g.w)
        for mask in range(1 << g.m):
            live = np.array([(mask >> e) & 1 for e in range(g.m)], dtype=bool)
            pr = float(np.prod(np.where(live, p, 1 - p)))
            A = np.zeros((n, n), dtype=np.int64)
            A[src[live], g.dst[live]] = 1
            R = np.eye(n, dtype=bool)
            for _ in range(n):
                R = R | (R.astype(np.int64) @ A > 0)
            out.append((pr, R))
        return out
    ins = [[] for _ in range(n)]
    for e in range(g.m):
        ins[g.dst[e]].append(e)
    choices = []
    for v in range(n):
        es = sorted(ins[v], key=lambda e: src[e])
        acc = np.float32(0)
        prev = 0.0
        opts = []
        for e in es:
            acc = np.float32(acc + g.w[e])
            t = min(math.ceil(float(acc) * 2 ** 24), 2 ** 24) / 2 ** 24
            opts.append((src[e], t - prev))
            prev = t
        opts.append((None, 1.0 - prev))
        choices.append(opts)
    for combo in itertools.product(*choices):
        pr = float(np.prod([c[1] for c in combo]))
        if pr == 0:
            continue
        R = np.zeros((n, n), dtype=bool)
        for v in range(n):
            seen = {v}
            cur = v
            while True:
                s = combo[cur][0]
                if s is None or s in seen:
                    break
                seen.add(s)
                cur = s
            for u in seen:
                R[u, v] = True
        out.append((pr, R))
    return out


def test_wc_matches_enumeration(orc):
    """Weighted cascade: p(u,v) = 1/indeg(v); compare membership with enumeration."""
    g = G.tiny_graph(6, 11, 21)
    indeg = g.indeg()
    w = (1.0 / indeg[g.dst]).astype(np.float32)
    gw = G.with_weights(g, w)
    P = _exact_ic_member_prob(gw)
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    theta = 100_000
    st = orc.sample_store(og, 77, theta)
    cnt = st.counts(g.n).astype(np.float64)
    pu = P.mean(axis=1)
    z = (cnt - theta * pu) / np.sqrt(theta * pu * (1 - pu) + 1e-12)
    assert np.all(np.abs(z) < 5), z


# ---------------------------------------------------------------- greedy
def _random_sets(rng, n, ns, maxlen):
    sets = []
    for _ in range(ns):
        k = rng.integers(1, maxlen + 1)
        sets.append(np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int32))
    off = np.zeros(ns + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in sets])
    return sets, off, np.concatenate(sets).astype(np.int32)


@pytest.mark.parametrize("seed", range(6))
def test_greedy_against_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    n, ns, k = 9, 40, 3
    sets, off, mem = _random_sets(rng, n, ns, 4)
    seeds, gains, cov = orc.greedy_sets(off, mem, n, k)
    # marginal gains from the definition, and argmax with lowest-id ties
    covered = np.zeros(ns, dtype=bool)
    for t in range(k):
        marg = np.array([sum(1 for j in range(ns) if not covered[j] and v in sets[j]) for v in range(n)])
        marg_sel = marg.copy()
        marg_sel[list(seeds[:t])] = -1
        assert seeds[t] == int(np.argmax(marg_sel))
        assert gains[t] == marg[seeds[t]]
        for j in range(ns):
            if seeds[t] in sets[j]:
                covered[j] = True
    assert cov == covered.sum() == int(gains.sum())
    assert np.all(np.diff(gains.astype(np.int64)) <= 0)
    # (1 - 1/e) bound against the optimum over all k-subsets
    best = 0
    for S in itertools.combinations(range(n), k):
        best = max(best, sum(1 for s in sets if set(S) & set(s.tolist())))
    assert cov >= (1 - 1 / math.e) * best


def test_greedy_zero_gain_and_k_equals_n(orc):
    off = np.array([0, 1, 2], dtype=np.int64)
    mem = np.array([3, 3], dtype=np.int32)
    seeds, gains, cov = orc.greedy_sets(off, mem, 5, 5)
    assert list(seeds) == [3, 0, 1, 2, 4] and list(gains) == [2, 0, 0, 0, 0] and cov == 2
    with pytest.raises(ValueError):
        orc.greedy_sets(off, mem, 5, 6)


# ---------------------------------------------------------------- IMM
def test_theta_matches_eq1(orc):
    """theta_i from the printed Eq. 1, read with '+ l *' for the garbled product."""
    for n, k, eps, l in [(1 << 20, 50, 0.5, 1.0), (1 << 23, 100, 0.13, 1.0), (4096, 5, 0.3, 1.0)]:
        prm = orc.imm_params(n, k, eps, l)
        la = l * (1 + math.log(2) / math.log(n))
        logC = math.lgamma(n + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1)
        for i in (1, 2, 5):
            eq1 = (2 + 2 * math.sqrt(2) / 3 * eps) * (logC + la * math.log(n) + math.log(math.log2(n))) * 2 ** i / (
                2 * eps ** 2)
            th = prm["lambda_prime"] / (n / 2 ** i)
            assert th == pytest.approx(eq1, rel=1e-9)


def test_imm_rounds_double(orc):
    g = G.rmat(11, seed=3)
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    seeds, gains, st, store = orc.imm(og, 5, 0.5, 1.0, 42)
    th = st["theta_round"]
    for a, b in zip(th, th[1:]):
        assert abs(b - 2 * a) <= 1
    assert store.nsets == max(st["theta_final"], th[-1])
    # final greedy agrees with a fresh greedy over the same store
    s2, g2, c2 = orc.greedy(store, g.n, 5)
    assert list(s2) == list(seeds) and c2 == st["coverage"]


def test_imm_approximation_on_tiny_graph(orc):
    g = _tiny(8, n=6, m=10)
    og = orc.Graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
    worlds = _exact_reach_table(g, False)

    def infl(S):
        return sum(pr * R[list(S), :].any(axis=0).sum() for pr, R in worlds)

    k, eps = 2, 0.3
    seeds, gains, st, _ = orc.imm(og, k, eps, 1.0, 5)
    opt = max(infl(S) for S in itertools.combinations(range(g.n), k))
    assert infl(seeds.tolist()) >= (1 - 1 / math.e - eps) * opt


def _tang_params(n, k, eps, l):
    """lambda' and lambda* of Tang, Shi and Xiao (SIGMOD 2015), written from their definitions by a
    route of its own: ln C(n, k) from the exact integer binomial (math.comb), l adjusted to
    l (1 + ln 2 / ln n) so that the whole run fails with probability at most 1/n^l (their
    Section 3.3), eps' = sqrt(2) eps in the sampling phase, and
      lambda' = (2 + 2 eps'/3) (ln C(n,k) + l ln n + ln log2 n) n / eps'^2          (phase 1)
      alpha   = sqrt(l ln n + ln 2),  beta = sqrt((1 - 1/e)(ln C(n,k) + l ln n + ln 2))
      lambda* = 2 n ((1 - 1/e) alpha + beta)^2 / eps^2                              (phase 2)."""
    lnn = math.log(n)
    la = l * (1.0 + math.log(2.0) / lnn)
    lnc = math.log(math.comb(n, k))
    ep = math.sqrt(2.0) * eps
    lam_p = (2.0 + 2.0 * ep / 3.0) * (lnc + la * lnn + math.log(math.log2(n))) * n / ep ** 2
    e1 = 1.0 - math.exp(-1.0)
    alpha = math.sqrt(la * lnn + math.log(2.0))
    beta = math.sqrt(e1 * (lnc + la * lnn + math.log(2.0)))
    lam_s = 2.0 * n * (e1 * alpha + beta) ** 2 / eps ** 2
    return lam_p, lam_s


@pytest.mark.parametrize("n,k,eps,l", [(1 << 20, 50, 0.5, 1.0), (1 << 23, 100, 0.13, 1.0), (4096, 5, 0.3, 1.0),
                                       (41_700_000, 200, 0.2, 1.0), (64, 3, 0.7, 2.0)])
def test_lambda_star_independent(orc, n, k, eps, l):
    """The oracle's lambda' and lambda* against Tang et al.'s definitions evaluated independently."""
    prm = orc.imm_params(n, k, eps, l)
    lam_p, lam_s = _tang_params(n, k, eps, l)
    assert prm["lambda_prime"] == pytest.approx(lam_p, rel=1e-9)
    assert prm["lambda_star"] == pytest.approx(lam_s, rel=1e-9)
    assert prm["eps_prime"] == pytest.approx(math.sqrt(2) * eps, rel=1e-15)


def test_lambda_star_eps_scaling(orc):
    """alpha and beta do not depend on eps, so lambda*(eps/2) = 4 lambda*(eps) exactly (halving eps
    quarters eps^2 by a power of two; no rounding differs)."""
    for n, k, eps in [(1 << 20, 50, 0.5), (1 << 23, 100, 0.26), (5000, 7, 0.3)]:
        a = orc.imm_params(n, k, eps, 1.0)["lambda_star"]
        b = orc.imm_params(n, k, eps / 2, 1.0)["lambda_star"]
        assert b == 4.0 * a


def _independent_imm_k1(n, sets_of, k_eps_l):
    """IMM's two phases (Tang et al.) for k = 1, driven independently of the oracle's driver: the
    RR sets come from `sets_of(theta)`; the greedy pick for k = 1 is the vertex in most sets
    (lowest id on ties); the stop test of round i is n cov_i / theta_i >= (1 + eps') n / 2^i."""
    k, eps, l = k_eps_l
    lam_p, lam_s = _tang_params(n, k, eps, l)
    ep = math.sqrt(2.0) * eps
    lb, rounds = 1.0, []
    i = 1
    while i <= math.log2(n) - 1:
        x = n / 2.0 ** i
        th = math.ceil(lam_p / x)
        cnt = np.zeros(n, dtype=np.int64)
        for s in sets_of(th):
            cnt[s] += 1
        cov = int(cnt.max())
        rounds.append((th, cov))
        if n * cov / th >= (1.0 + ep) * x:
            lb = n * cov / (th * (1.0 + ep))
            break
        i += 1
    return rounds, lb, math.ceil(lam_s / lb)


def test_imm_all_live_star_round_one(orc):
    """Every edge 0 -> v live: each RR set holds vertex 0, seed {0} covers every set, so the
    first round passes its test (n >= (1 + eps') n / 2 for eps <= 1/sqrt 2) with
    LB = n / (1 + sqrt(2) eps) exactly, and theta = ceil(lambda* (1 + sqrt(2) eps) / n)."""
    n = 2048
    g = G._csr_from_pairs(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))
    og = orc.Graph(n, g.row_ptr, g.dst, np.ones(g.m, dtype=np.float32), model="IC", prob="EDGE")
    for eps in (0.5, 0.3, 0.7):
        seeds, gains, st, store = orc.imm(og, 1, eps, 1.0, 11)
        ep = math.sqrt(2.0) * eps
        lam_p, lam_s = _tang_params(n, 1, eps, 1.0)
        assert st["rounds"] == 1
        assert st["theta_round"][0] == math.ceil(lam_p / (n / 2))
        assert st["cov_round"][0] == st["theta_round"][0]
        assert st["lb"] == pytest.approx(n / (1.0 + ep), rel=1e-12)
        assert -1e-6 < st["theta_final"] - lam_s * (1.0 + ep) / n < 1.0 + 1e-6
        assert list(seeds) == [0] and st["coverage"] == st["nsets_final"]
        assert st["nsets_final"] == max(st["theta_final"], st["theta_round"][0])


def test_imm_partial_star_later_round(orc):
    """Edges 0 -> v live for v < n/8 only: vertex 0 is in the sets rooted below n/8, so the best
    single seed covers about 1/8 of the sets and the stop test first passes in round 4 for
    eps = 0.5.  The oracle's rounds, coverage, LB and final theta equal an independent driver's
    over the oracle's own (separately pinned) RR sets."""
    n, a = 4096, 4096 // 8
    g = G._csr_from_pairs(n, np.zeros(a - 1, dtype=np.int64), np.arange(1, a))
    og = orc.Graph(n, g.row_ptr, g.dst, np.ones(g.m, dtype=np.float32), model="IC", prob="EDGE")
    seed = 21
    for eps in (0.5, 0.35):
        seeds, gains, st, store = orc.imm(og, 1, eps, 1.0, seed)
        rounds, lb, theta = _independent_imm_k1(n, lambda th: [og.sample(seed, j) for j in range(th)],
                                                (1, eps, 1.0))
        assert [(t, c) for t, c in zip(st["theta_round"], st["cov_round"])] == rounds
        assert st["lb"] == pytest.approx(lb, rel=1e-12)
        assert abs(st["theta_final"] - theta) <= 1
        if eps == 0.5:
            assert st["rounds"] == 4


# ---------------------------------------------------------------- Huffman
def _heap_cost(w):
    import heapq

    h = [int(x) for x in w if x > 0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("seed", range(5))
def test_huffman_optimal_and_kraft(orc, seed):
    rng = np.random.default_rng(seed)
    w = rng.zipf(1.6, size=300).astype(np.uint64)
    w[rng.random(300) < 0.3] = 0
    lens = orc.huffman_lengths(w)
    assert np.all((lens > 0) == (w > 0))
    assert sum(2.0 ** -int(L) for L in lens if L) == pytest.approx(1.0, abs=1e-12)
    assert int((lens.astype(np.uint64) * w).sum()) == _heap_cost(w)
    codes = orc.canonical_codes(lens)
    words = {format(int(c), f"0{int(L)}b") for c, L in zip(codes, lens) if L}
    assert len(words) == int((lens > 0).sum())
    for a in words:  # prefix-free
        for b in words:
            assert a == b or not b.startswith(a)


def test_huffman_length_limit_and_single(orc):
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    lens = orc.huffman_lengths(np.array(fib, dtype=np.uint64))
    assert lens.max() <= 32
    assert sum(2.0 ** -int(L) for L in lens) == pytest.approx(1.0)
    one = orc.huffman_lengths(np.array([0, 0, 5, 0], dtype=np.uint64))
    assert list(one) == [0, 0, 1, 0]


@pytest.mark.parametrize("enc", ["NONE", "HUFFMAN", "HOT_BITMAP", "HUFFMAN_HOT_BITMAP"])
@pytest.mark.parametrize("model", ["IC", "LT"])
def test_encode_roundtrip(orc, enc, model):
    g = G.rmat(10, seed=4)
    w = G.lt_weights(g, 9) if model == "LT" else None
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob="WC" if model == "IC" else "EDGE")
    theta = 1500
    st = orc.sample_store(og, 42, theta)
    W = orc.warmup_count(0.1, theta)
    e = orc.Encoded(st, g.n, enc, W, hot_frac=0.01)
    off, mem = st.arrays()
    for j in range(theta):
        assert np.array_equal(e.decode_set(j), mem[off[j]:off[j + 1]])
    if enc in ("HUFFMAN", "HUFFMAN_HOT_BITMAP"):
        warm = st.counts(g.n, 0, W)
        hot = set(e.hot.tolist())
        alph = [v for v in range(g.n) if warm[v] > 0 and v not in hot]
        assert set(np.nonzero(e.lens)[0].tolist()) == set(alph)
        # payload = gamma count + verbatim ids + code lengths, summed over all sets
        tot = 0
        for j in range(theta):
            s = [v for v in mem[off[j]:off[j + 1]] if v not in hot]
            nesc = sum(1 for v in s if e.lens[v] == 0)
            tot += 2 * int(math.floor(math.log2(nesc + 1))) + 1 + nesc * e.wbits + sum(int(e.lens[v]) for v in s)
        assert tot == e.payload_bits
    if enc in ("HOT_BITMAP", "HUFFMAN_HOT_BITMAP"):
        warm = st.counts(g.n, 0, W)
        order = sorted([v for v in range(g.n) if warm[v] > 0], key=lambda v: (-int(warm[v]), v))
        assert list(e.hot) == order[:math.ceil(0.01 * g.n)]
        full = st.counts(g.n)
        for r, v in enumerate(e.hot):
            pc = sum(bin(int(e.bitmap[wd * e.nhot + r])).count("1") for wd in range(e.nwords))
            assert pc == full[v]


@pytest.mark.parametrize("dens", [0.0, 1.0 / 32, 0.25, 1.0])
def test_hot_density_gate(orc, dens):
    """The gated hot set holds exactly the top vertices among those in at least
    ceil(dens * W) warm-up sets, its rows are cheaper than 32-bit ids once dens >= 1/32,
    and decoding still gives back every set."""
    g = G.rmat(10, seed=5)
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    theta = 2000
    st = orc.sample_store(og, 42, theta)
    W = orc.warmup_count(0.2, theta)
    e = orc.Encoded(st, g.n, "HUFFMAN_HOT_BITMAP", W, hot_frac=0.05, hot_min_density=dens)
    warm = st.counts(g.n, 0, W)
    thr = max(1, math.ceil(dens * W))
    eligible = sorted([v for v in range(g.n) if warm[v] >= thr], key=lambda v: (-int(warm[v]), v))
    assert list(e.hot) == eligible[:math.ceil(0.05 * g.n)]
    if dens >= 1.0 / 32:
        # each row (one bit per warm-up set) costs no more than the vertex's ids would
        assert all(W <= 32 * int(warm[v]) for v in e.hot)
    off, mem = st.arrays()
    for j in range(0, theta, 7):
        assert np.array_equal(e.decode_set(j), mem[off[j]:off[j + 1]])


def _stream_order(e, j):
    """Members of encoded set j in stream order: (escaped ids, coded ids), read bit by bit."""
    pay = e.payload
    bit = lambda p: (int(pay[p >> 5]) >> (31 - (p & 31))) & 1
    pos, end = int(e.bitoff[j]), int(e.bitoff[j + 1])
    L = 0
    while bit(pos) == 0:
        L, pos = L + 1, pos + 1
    g = 0
    for _ in range(L + 1):
        g, pos = (g << 1) | bit(pos), pos + 1
    esc = []
    for _ in range(g - 1):
        v = 0
        for _ in range(e.wbits):
            v, pos = (v << 1) | bit(pos), pos + 1
        esc.append(v)
    book = {(int(e.lens[v]), int(e.codes[v])): v for v in np.nonzero(e.lens)[0]}
    coded = []
    while pos < end:
        c, ln = 0, 0
        while (ln, c) not in book:
            c, ln, pos = (c << 1) | bit(pos), ln + 1, pos + 1
            assert ln <= 32
        coded.append(book[(ln, c)])
    return esc, coded


@pytest.mark.parametrize("model", ["IC", "LT"])
def test_huffman_string_order(orc, model):
    """Escaped ids ascend; u*_enc (the warm-up top vertex) leads the coded part; the other codes
    follow in canonical order, i.e. by (code length, id)."""
    g = G.rmat(10, seed=6)
    w = G.lt_weights(g, 9) if model == "LT" else None
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob="WC" if model == "IC" else "EDGE")
    theta = 800
    st = orc.sample_store(og, 42, theta)
    W = orc.warmup_count(0.1, theta)
    e = orc.Encoded(st, g.n, "HUFFMAN", W)
    warm = st.counts(g.n, 0, W)
    assert e.ustar_enc == int(np.argmax(warm))  # most frequent, lowest id on ties
    off, mem = st.arrays()
    fronts = 0
    for j in range(theta):
        esc, coded = _stream_order(e, j)
        assert sorted(esc + coded) == list(mem[off[j]:off[j + 1]])
        assert esc == sorted(esc) and all(e.lens[v] == 0 for v in esc)
        rest = coded
        if e.ustar_enc in coded:
            assert coded[0] == e.ustar_enc
            rest = coded[1:]
            fronts += 1
        keys = [(int(e.lens[v]), int(v)) for v in rest]
        assert keys == sorted(keys)
    assert fronts > 0


def test_characterize_eq2(orc):
    g = G.rmat(10, seed=4)
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    st = orc.sample_store(og, 42, 3000)
    off, _ = st.arrays()
    X = np.diff(off).astype(np.float64)
    S, D = st.characterize(g.n, 0, 3000)
    assert S == pytest.approx(scipy.stats.skew(X, bias=True), rel=1e-9)
    assert D == pytest.approx(X.sum() / (3000 * g.n), rel=1e-12)


def test_in_csr_sorted(orc):
    g = G.rmat(10, seed=6)
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    ptr, src = og.in_csr()
    assert np.array_equal(ptr, np.concatenate([[0], np.cumsum(g.indeg())]))
    for v in range(g.n):
        row = src[ptr[v]:ptr[v + 1]]
        assert np.all(np.diff(row) > 0)
    # every forward edge appears exactly once
    fwd = set(zip(g.src().tolist(), g.dst.tolist()))
    rev = {(int(u), v) for v in range(g.n) for u in src[ptr[v]:ptr[v + 1]]}
    assert fwd == rev


def test_append_range_shards_equal_the_store(orc):
    """Shards of the index range, appended to stores of their own, concatenate to the store
    a plain extend builds (the benchmark times the oracle this way on several threads)."""
    from synth import graphs as G

    g = G.erdos_renyi(300, 2400, seed=4, p_hi=0.4)
    og = orc.Graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
    whole = orc.sample_store(og, 9, 1000)
    woff, wmem = whole.arrays()
    parts = []
    for j0, j1 in ((0, 137), (137, 600), (600, 1000)):
        s = orc.Store()
        s.append_range(og, 9, j0, j1)
        off, mem = s.arrays()
        assert s.nsets == j1 - j0
        assert np.array_equal(off, woff[j0:j1 + 1] - woff[j0])
        parts.append(mem.copy())
    assert np.array_equal(np.concatenate(parts), wmem)


# ---------------------------------------------------------------- Bitmax (all vertices) and Alg. 1's choice
def test_bitmax_eq3_rows_and_subtract(orc):
    """The worked example of Eq. 3 through the all-vertex Bitmax store and Alg. 3: the rows
    are the printed left matrix; after the first pick (v1) the rows are the printed right
    matrix."""
    before, after, first = _eq3()
    off, mem = _sets_from_rows(before)
    st = orc.Store.from_sets(off, mem)
    e = orc.Encoded(st, 5, "BITMAX", W=6)
    assert e.enc_name == "BITMAX" and e.nhot == 5 and list(e.hot) == [0, 1, 2, 3, 4] and e.nwords == 1
    for v in range(5):
        assert [(int(e.bitmap[v]) >> j) & 1 for j in range(6)] == list(before[v])
    seeds, gains, cov, rows = e.bitmax_select(1, want_after=True)
    assert seeds[0] == first and gains[0] == before[first].sum() and cov == gains[0]
    for v in range(5):
        assert [(int(rows[v]) >> j) & 1 for j in range(6)] == list(after[v])


@pytest.mark.parametrize("model", ["IC", "LT"])
def test_bitmax_round_trip_and_alg3_equals_greedy(orc, model):
    """decode(encode(R)) == R for the all-vertex bit matrix (column padding to 64 adds no
    member), and Alg. 3 on the matrix picks exactly the plain greedy's seeds and gains, for
    every k up to n (zero-gain picks included)."""
    g = G.rmat(8, seed=11)
    w = G.lt_weights(g, 5) if model == "LT" else np.full(g.m, 0.2, dtype=np.float32)
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob="EDGE")
    st = orc.sample_store(og, 17, 1000)  # 1000 sets: the last word is padded
    off, mem = st.arrays()
    e = orc.Encoded(st, g.n, "BITMAX", W=100)
    assert e.nwords == 16
    for j in range(st.nsets):
        assert np.array_equal(e.decode_set(j), mem[off[j]:off[j + 1]])
    for k in (1, 7, 40, g.n):
        s1, g1, c1 = e.bitmax_select(k)
        s2, g2, c2 = orc.greedy(st, g.n, k)
        assert np.array_equal(s1, s2) and np.array_equal(g1, g2) and c1 == c2


def _sizes_store(orc, sizes, n, seed=0):
    """A store whose sets have the given sizes (members drawn without replacement)."""
    rng = np.random.default_rng(seed)
    sets = [np.sort(rng.choice(n, size=int(s), replace=False)).astype(np.int32) for s in sizes]
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(x) for x in sets])
    return orc.Store.from_sets(off, np.concatenate(sets).astype(np.int32))


def test_auto_choice_follows_skewness_and_density(orc):
    """Alg. 1 with the Bitmax encoding paragraph: Bitmax exactly when Eq. 2's skewness of the
    first block is negative and its density is above 1/32; otherwise Huffmax.  The skewness
    sign and the density are checked against scipy on the same sizes."""
    from scipy import stats

    n = 400
    left = [300] * 90 + [5] * 10         # long left tail: S < 0, D ~ 0.68
    right = [5] * 90 + [300] * 10        # long right tail: S > 0, D ~ 0.09
    thin = [12] * 90 + [1] * 10          # S < 0 but D = 0.027 <= 1/32
    for sizes, want in ((left, "BITMAX"), (right, "HUFFMAN"), (thin, "HUFFMAN")):
        st = _sizes_store(orc, sizes, n)
        S, D = st.characterize(n, 0, len(sizes))
        assert np.sign(S) == np.sign(stats.skew(sizes)) and D == pytest.approx(sum(sizes) / (len(sizes) * n))
        e = orc.Encoded(st, n, "AUTO", W=len(sizes))
        assert e.enc_name == want, (S, D)
        for j in (0, len(sizes) - 1):
            assert np.array_equal(e.decode_set(j), st.arrays()[1][st.arrays()[0][j]:st.arrays()[0][j + 1]])
    # the density boundary itself: D exactly 1/32 stays Huffmax (Bitmax needs D > 1/32), one
    # vertex fewer tips it over
    sizes = [5] * 15 + [1]
    for n, want in ((152, "HUFFMAN"), (151, "BITMAX")):
        st = _sizes_store(orc, sizes, n)
        S, D = st.characterize(n, 0, len(sizes))
        assert S < 0 and (D == 1.0 / 32) == (n == 152)
        assert orc.Encoded(st, n, "AUTO", W=len(sizes)).enc_name == want


def test_append_range_threads_with_own_scratch(orc):
    """Shards sampled at once on several threads, each with its own scratch, are the same sets
    as one thread's (the sampling scratch is the only mutable state a sample touches)."""
    import threading

    from synth import graphs as G

    g = G.erdos_renyi(2000, 32000, seed=7, p_hi=0.2)
    og = orc.Graph(g.n, g.row_ptr, g.dst, g.w, model="IC", prob="EDGE")
    whole = orc.sample_store(og, 3, 4000)
    woff, wmem = whole.arrays()
    parts = [None] * 8

    def work(t):
        sc = orc.Scratch(g.n)
        s = orc.Store()
        s.append_range(og, 3, t * 500, (t + 1) * 500, sc)
        parts[t] = s

    ts = [threading.Thread(target=work, args=(t,)) for t in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    mems = [p.arrays()[1].copy() for p in parts]
    assert sum(p.nsets for p in parts) == 4000
    assert np.array_equal(np.concatenate(mems), wmem)


# ---------------------------------------------------------------- implicit roots
@pytest.mark.parametrize("model", ["IC", "LT"])
@pytest.mark.parametrize("enc", ["NONE", "HUFFMAN", "HOT_BITMAP", "HUFFMAN_HOT_BITMAP", "BITMAX"])
def test_implicit_roots_round_trip_and_saving(orc, model, enc):
    """Every set holds its root, a function of (seed, j): dropping it from the stored part and
    regenerating it on decode gives back every set, and saves exactly the root's own cost in
    each set where it is not in a bitmap row (4 bytes as a plain id; its code, or its escape
    and the longer escape count, in a Huffman string)."""
    g = G.rmat(9, seed=12)
    w = G.lt_weights(g, 6) if model == "LT" else None
    og = orc.Graph(g.n, g.row_ptr, g.dst, w, model=model, prob="EDGE" if model == "LT" else "WC")
    st = orc.sample_store(og, 23, 3000)
    off, mem = st.arrays()
    ex = orc.Encoded(st, g.n, enc, W=300, hot_frac=0.02)
    im = orc.Encoded(st, g.n, enc, W=300, hot_frac=0.02, implicit_roots=True)
    for j in range(0, 3000, 7):
        assert np.array_equal(im.decode_set(j), mem[off[j]:off[j + 1]])
    roots = np.array([orc.root(g.n, 23, j) for j in range(3000)])
    hot = set(ex.hot.tolist()) if ex.nhot else set()
    cold = np.array([r not in hot for r in roots])
    if enc in ("NONE", "HOT_BITMAP"):
        assert ex.cold_off[-1] - im.cold_off[-1] == cold.sum()
    elif enc == "BITMAX":
        assert cold.sum() == 0 and np.array_equal(ex.bitmap, im.bitmap)
    else:
        gam = lambda x: 2 * int(np.floor(np.log2(x))) + 1
        saved = 0
        for j in range(3000):
            r = int(roots[j])
            if not cold[j]:
                continue
            if ex.lens[r]:
                saved += int(ex.lens[r])
            else:
                nesc = sum(1 for v in mem[off[j]:off[j + 1]] if v not in hot and ex.lens[v] == 0)
                saved += ex.wbits + gam(nesc + 1) - gam(nesc)
        assert ex.payload_bits - im.payload_bits == saved


def test_implicit_roots_need_sampled_sets(orc):
    off = np.array([0, 2, 3], dtype=np.int64)
    st = orc.Store.from_sets(off, np.array([1, 2, 0], dtype=np.int32))
    with pytest.raises(ValueError):
        orc.Encoded(st, 4, "NONE", W=2, implicit_roots=True)


# ---------------------------------------------------------------- Roaring-style row containers
@pytest.mark.parametrize("enc", ["HOT_BITMAP", "HUFFMAN_HOT_BITMAP"])
@pytest.mark.parametrize("implicit", [False, True])
def test_row_containers(orc, enc, implicit):
    """Hot vertices below warm-up density 1/16 keep per 2^16-set chunk the sorted 16-bit
    offsets of their sets (array containers), the others bitmap rows: the split follows the
    rule, every list is strictly ascending and names exactly the sets that hold its vertex
    (over two chunks, the second partial), and every set decodes back, also with implicit
    roots."""
    g = G.rmat(10, seed=19)
    og = orc.Graph(g.n, g.row_ptr, g.dst, None, model="IC", prob="WC")
    T, W = 70_000, 3_000
    st = orc.sample_store(og, 4, T)
    off, mem = st.arrays()
    e = orc.Encoded(st, g.n, enc, W=W, hot_frac=0.05, implicit_roots=implicit, containers=True)
    plain = orc.Encoded(st, g.n, enc, W=W, hot_frac=0.05)
    warm = st.counts(g.n, 0, W)
    assert e.nar > 0 and e.nhot > 0 and e.nchunks == 2
    assert sorted(e.hot.tolist() + e.ar_hot.tolist()) == sorted(plain.hot.tolist())
    assert all(16 * warm[v] < W for v in e.ar_hot) and all(16 * warm[v] >= W for v in e.hot)
    assert [v for v in plain.hot if v in set(e.ar_hot.tolist())] == e.ar_hot.tolist()  # hot order kept
    sets_of = {int(v): [] for v in e.ar_hot}
    for j in range(T):
        for v in mem[off[j]:off[j + 1]]:
            if int(v) in sets_of:
                sets_of[int(v)].append(j)
    stride = e.nar + 1
    for a, v in enumerate(e.ar_hot):
        got = []
        for ch in range(e.nchunks):
            lo, hi = e.ar_off[ch * stride + a], e.ar_off[ch * stride + a + 1]
            seg = e.ar_low[lo:hi].astype(np.int64)
            assert (np.diff(seg) > 0).all()
            got += (seg + ch * 65536).tolist()
        assert got == sets_of[int(v)]
    assert len(e.ar_low) == sum(len(x) for x in sets_of.values())
    for j in list(range(0, T, 997)) + [65535, 65536, T - 1]:
        assert np.array_equal(e.decode_set(j), mem[off[j]:off[j + 1]])
