"""Seeded synthetic graphs shaped like the social networks the paper evaluates.

The paper measures on public graphs (DBLP ... twitter7, its Table of input
graphs); none of them is available here, so every workload is one of the
seeded synthetic families below, with the sizes and degree structure the
benchmark configurations name:

* ``erdos_renyi``  directed G(n, m) with distinct ordered pairs, no self-loops;
* ``rmat``         R-MAT (a, b, c, d) = (.57, .19, .19, .05), 16 * 2**scale samples,
                   seeded label permutation, self-loops and duplicates removed;
* ``chung_lu``     power-law digraph (exponent gamma) drawn source by source,
                   shaped like twitter7 (41.7M vertices, ~1.47B edges);
* ``flat_head``    G(n, m) with one constant IC probability: RR sets with a flat
                   head (negative skewness, high density), like the paper's
                   Bitmax graphs;
* ``lt_weights``   U(0,1) float32 in-weights rescaled so every vertex's in-weights
                   sum to at most 1 (rows whose sum exceeds 1 are divided by it).

Every generator returns a forward CSR: ``row_ptr`` int64[n+1], ``dst`` int32[m]
sorted ascending inside each row, and optional float32 weights ``w`` aligned with
``dst``.  Nothing here samples RR sets or selects seeds.
"""

from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    dst: np.ndarray  # int32 [m]
    w: Optional[np.ndarray] = None  # float32 [m] or None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.dst.shape[0])

    def src(self) -> np.ndarray:
        """Source id of every forward edge (int32[m])."""
        deg = np.diff(self.row_ptr)
        return np.repeat(np.arange(self.n, dtype=np.int32), deg)

    def indeg(self) -> np.ndarray:
        return np.bincount(self.dst, minlength=self.n).astype(np.int64)


def _csr_from_pairs(n: int, u: np.ndarray, v: np.ndarray, w=None, name=""):
    """Sort (u, v) pairs by (u, v), drop self-loops and duplicates, build CSR."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if w is not None:
        w = np.asarray(w)[keep]
    key = u * np.int64(n) + v
    if w is None:
        key = np.unique(key)
    else:
        key, first = np.unique(key, return_index=True)
        w = w[first].astype(np.float32)
    u = (key // n).astype(np.int64)
    dst = (key % n).astype(np.int32)
    counts = np.bincount(u, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, dst=dst, w=w, name=name)


def erdos_renyi(n: int, m: int, seed: int, p_hi: float = 0.1) -> Graph:
    """Directed G(n, m): m distinct ordered pairs (u != v), p ~ U[0, p_hi) float32."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(n * (n - 1), size=m, replace=False).astype(np.int64)
    u = idx // (n - 1)
    r = idx % (n - 1)
    v = r + (r >= u)
    order = np.lexsort((v, u))
    u, v = u[order], v[order]
    p = (rng.random(m, dtype=np.float32) * np.float32(p_hi)).astype(np.float32)
    g = _csr_from_pairs(n, u, v, p, name=f"er_n{n}_m{m}_s{seed}")
    assert g.m == m
    return g


def flat_head(n: int, m: int, p: float, seed: int) -> Graph:
    """Directed G(n, m) with one constant IC probability p on every edge: with mean live
    in-degree (m / n) * p well above 1 most roots reach a giant in-component, so RR-set
    sizes have a flat head and a short left tail (negative Eq. 2 skewness, density far
    above 1/32), the shape the paper reports for its Bitmax graphs."""
    g = erdos_renyi(n, m, seed=seed)
    g.w = np.full(g.m, p, dtype=np.float32)
    g.name = f"flat_n{n}_m{m}_p{p}_s{seed}"
    return g


def _cache_path(tag: str) -> Optional[str]:
    d = os.environ.get("HBM_GRAPH_CACHE", os.path.join(os.environ.get("TMPDIR", "/tmp"), "hbm_graph_cache"))
    try:
        os.makedirs(d, exist_ok=True)
    except OSError:
        return None
    h = hashlib.sha1(tag.encode()).hexdigest()[:16]
    return os.path.join(d, f"{h}.npz")


def _cached(tag: str, make):
    path = _cache_path(tag)
    if path is not None and os.path.exists(path):
        z = np.load(path)
        w = z["w"] if "w" in z.files else None
        return Graph(n=int(z["n"]), row_ptr=z["row_ptr"], dst=z["dst"], w=w, name=tag)
    g = make()
    if path is not None:
        tmp = path + f".tmp{os.getpid()}.npz"
        kw = dict(n=np.int64(g.n), row_ptr=g.row_ptr, dst=g.dst)
        if g.w is not None:
            kw["w"] = g.w
        np.savez(tmp, **kw)
        os.replace(tmp, path)
    return g


def rmat(scale: int, seed: int, edge_factor: int = 16, a=0.57, b=0.19, c=0.19, cache: bool = True) -> Graph:
    """R-MAT with 2**scale vertices and edge_factor * 2**scale samples.

    Each sample picks one quadrant per level; a seeded permutation relabels the
    vertices; self-loops and duplicates are removed afterwards.
    """
    n = 1 << scale
    M = edge_factor * n

    def make():
        rng = np.random.default_rng(seed)
        u = np.zeros(M, dtype=np.int32)
        v = np.zeros(M, dtype=np.int32)
        ab, abc = np.float32(a + b), np.float32(a + b + c)
        fa = np.float32(a)
        for _ in range(scale):
            r = rng.random(M, dtype=np.float32)
            ubit = r >= ab
            vbit = ((r >= fa) & (r < ab)) | (r >= abc)
            u <<= 1
            v <<= 1
            u |= ubit
            v |= vbit
            del r, ubit, vbit
        perm = rng.permutation(n).astype(np.int32)
        u = perm[u]
        v = perm[v]
        return _csr_from_pairs(n, u, v, None, name=f"rmat_s{scale}_ef{edge_factor}_seed{seed}")

    if cache and scale >= 16:
        return _cached(f"rmat:{scale}:{edge_factor}:{seed}:{a}:{b}:{c}", make)
    return make()


def lt_weights(g: Graph, seed: int) -> np.ndarray:
    """U(0,1) float32 in-weights; a vertex whose in-weights sum (in float64) above 1
    has each of them divided by that sum and rounded to float32."""
    rng = np.random.default_rng(seed)
    x = rng.random(g.m, dtype=np.float32)
    s = np.bincount(g.dst, weights=x.astype(np.float64), minlength=g.n)
    scale = np.where(s > 1.0, s, 1.0)
    return (x.astype(np.float64) / scale[g.dst]).astype(np.float32)


def with_weights(g: Graph, w: Optional[np.ndarray]) -> Graph:
    return Graph(n=g.n, row_ptr=g.row_ptr, dst=g.dst, w=w, name=g.name)


def tiny_graph(n: int, m: int, seed: int, p_lo=0.0, p_hi=1.0) -> Graph:
    """Small random digraph for exhaustive checks (distinct pairs, no self-loops)."""
    rng = np.random.default_rng(seed)
    m = min(m, n * (n - 1))
    idx = rng.choice(n * (n - 1), size=m, replace=False).astype(np.int64)
    u = idx // (n - 1)
    r = idx % (n - 1)
    v = r + (r >= u)
    p = (p_lo + (p_hi - p_lo) * rng.random(m)).astype(np.float32)
    return _csr_from_pairs(n, u, v, p, name=f"tiny_n{n}_m{m}_s{seed}")


def chung_lu_csr(n: int, avg_deg: float, gamma: float, seed: int, max_deg: float, device: str = "cpu",
                 chunk: int = 1 << 22):
    """Chung-Lu power-law digraph as a forward CSR of torch tensors on ``device``.

    Out- and in-weights are proportional to (i + i0)^(-1/(gamma-1)), permuted
    independently; i0 is chosen so the largest expected degree is about
    ``max_deg`` (the expected edge count is avg_deg * n).  Source by source,
    each vertex draws a Poisson out-degree with mean proportional to its
    out-weight, then that many targets with probability proportional to
    in-weight; duplicates and self-loops are dropped, so rows come out sorted
    and the CSR needs no global sort.  Deterministic for a seed and device type.
    Returns (row_ptr int64[n+1], dst int32[m]).
    """
    import torch

    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    expo = 1.0 / (gamma - 1.0)
    idx = torch.arange(n, dtype=torch.float64, device=dev)
    m_target = avg_deg * n
    lo, hi = 1e-3, float(n)
    for _ in range(80):  # i0 by bisection: the top expected degree ~= max_deg
        mid = (lo * hi) ** 0.5
        wv = (idx + mid) ** (-expo)
        if float(m_target * wv[0] / wv.sum()) > max_deg:
            lo = mid
        else:
            hi = mid
    wv = (idx + hi) ** (-expo)
    del idx
    p_out = torch.randperm(n, generator=gen, device=dev)
    p_in = torch.randperm(n, generator=gen, device=dev)
    w_out = torch.empty_like(wv)
    w_out[p_out] = wv
    w_in = torch.empty_like(wv)
    w_in[p_in] = wv
    del wv, p_out, p_in
    lam = m_target * w_out / w_out.sum()
    cdf = torch.cumsum(w_in / w_in.sum(), 0)
    cdf[-1] = 1.0
    del w_in, w_out
    outdeg = torch.poisson(lam, generator=gen).to(torch.int64)
    del lam
    counts = torch.zeros(n, dtype=torch.int64, device=dev)
    dsts = []
    cum = torch.cumsum(outdeg, 0)
    v0 = 0
    while v0 < n:
        base = int(cum[v0 - 1].item()) if v0 else 0
        v1 = int(torch.searchsorted(cum, torch.tensor(base + chunk, device=dev, dtype=torch.int64)).item()) + 1
        v1 = min(max(v1, v0 + 1), n)
        d = outdeg[v0:v1]
        tot = int(d.sum().item())
        if tot:
            r = torch.rand(tot, generator=gen, device=dev, dtype=torch.float64)
            t = torch.searchsorted(cdf, r).clamp_(max=n - 1)
            s = torch.repeat_interleave(torch.arange(v0, v1, device=dev, dtype=torch.int64), d)
            keep = s != t
            key = torch.unique(s[keep] * n + t[keep])  # sorted by (source, target)
            counts[v0:v1] = torch.bincount(key // n - v0, minlength=v1 - v0)
            dsts.append((key % n).to(torch.int32))
            del r, t, s, keep, key
        v0 = v1
    dst = torch.cat(dsts) if dsts else torch.zeros(0, dtype=torch.int32, device=dev)
    del dsts
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(counts, 0, out=row_ptr[1:])
    return row_ptr, dst


def chung_lu(n: int, avg_deg: float, gamma: float, seed: int, max_deg: float, device: str = "cpu",
             chunk: int = 1 << 22) -> Graph:
    """``chung_lu_csr`` as a host Graph (numpy arrays)."""
    row_ptr, dst = chung_lu_csr(n, avg_deg, gamma, seed, max_deg, device=device, chunk=chunk)
    return Graph(n=n, row_ptr=row_ptr.cpu().numpy(), dst=dst.cpu().numpy(), w=None,
                 name=f"chunglu_n{n}_g{gamma}_s{seed}")


# ----------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# ----------------------------------------------------------------------------

CONFIGS = {
    # tiny IC instance: ER n=1024, m=8192, p~U[0,0.1], theta=10^4, k=10, seed 42
    "c1": dict(kind="er", n=1024, m=8192, gseed=1, model="IC", prob="EDGE", theta=10_000, k=10,
               seed=42, enc="NONE"),
    # IMM under IC weighted cascade on R-MAT scale 20, eps=.5, l=1, k=50, hot bitmap 1% from 10% warm-up
    "c2": dict(kind="rmat", scale=20, gseed=2, model="IC", prob="WC", eps=0.5, l=1.0, k=50, seed=42,
               enc="HOT_BITMAP", warmup=0.10, hot=0.01),
    # flat-head IC (Bitmax-shaped): G(65536, 2^20) with p = 0.1 on every edge, eps=.5, k=50,
    # encoding chosen by Alg. 1 from a 10% warm-up
    "flat": dict(kind="flat", n=65536, m=1 << 20, p=0.1, gseed=6, model="IC", prob="EDGE", eps=0.5, l=1.0, k=50,
                 seed=42, enc="AUTO", warmup=0.10, hot=0.01),
    # IMM under LT on R-MAT scale 23, eps=.13, k=100, Huffman from 5% warm-up
    "c3": dict(kind="rmat", scale=23, gseed=3, model="LT", prob="EDGE", eps=0.13, l=1.0, k=100, seed=42,
               enc="HUFFMAN", warmup=0.05, hot=0.0),
}


# the served graph: Chung-Lu shaped like twitter7 (41,652,230 vertices, 1,468,365,182 edges,
# largest degree 770,155), exponent 2.2, weighted cascade; queries k ~ U{10..200}, eps in {.5, .2}
C5 = dict(n=41_700_000, avg_deg=1_468_365_182 / 41_652_230, gamma=2.2, max_deg=770_155, gseed=5,
          model="IC", prob="WC", enc="HUFFMAN_HOT_BITMAP", warmup=0.05, hot=0.01, hot_density=1.0 / 32,
          budget=200 * 10 ** 9)


QUERY_POOL = 4096


def serving_queries(count: int, seed: int = 5, rate: float = 1.0):
    """Poisson arrivals (mean gap 1/rate seconds) of IMM queries: k ~ U{10..200}, eps in
    {.5, .2}, l = 1, sampling seed 1000 + q.  Query q is the same for every count (up to
    QUERY_POOL queries are drawn, then cut) and every rate (the gaps scale with 1/rate)."""
    N = max(count, QUERY_POOL)
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=N)[:count]
    ks = rng.integers(10, 201, size=N)
    eps = rng.choice(np.array([0.5, 0.2]), size=N)
    t = np.cumsum(gaps) - gaps[0]
    return [dict(q=q, t=float(t[q]), k=int(ks[q]), eps=float(eps[q]), l=1.0, seed=1000 + q) for q in range(count)]


def config_graph(name: str, scale_override: Optional[int] = None) -> Graph:
    c = CONFIGS[name]
    if c["kind"] == "er":
        return erdos_renyi(c["n"], c["m"], seed=c["gseed"])
    if c["kind"] == "flat":
        return flat_head(c["n"], c["m"], c["p"], seed=c["gseed"])
    scale = scale_override if scale_override is not None else c["scale"]
    g = rmat(scale, seed=c["gseed"])
    if c["model"] == "LT":
        g = with_weights(g, lt_weights(g, seed=c["gseed"] + 100))
    return g


def batched_instances(count: int = 256, seed: int = 4, smin: int = 12, smax: int = 18):
    """Parameters of the batched workload: scale ~ U{smin..smax}, IC-WC for even
    instances and LT for odd ones, k ~ U{5..100}, eps in {.5, .3}, sampling seed 42+i."""
    rng = np.random.default_rng(seed)
    scales = rng.integers(smin, smax + 1, size=count)
    ks = rng.integers(5, 101, size=count)
    eps = rng.choice(np.array([0.5, 0.3]), size=count)
    out = []
    for i in range(count):
        model = "IC" if i % 2 == 0 else "LT"
        out.append(dict(index=i, scale=int(scales[i]), model=model, prob="WC" if model == "IC" else "EDGE",
                        k=int(ks[i]), eps=float(eps[i]), l=1.0, seed=42 + i, gseed=1000 + i,
                        enc="HOT_BITMAP" if model == "IC" else "HUFFMAN",
                        warmup=0.10 if model == "IC" else 0.05, hot=0.01 if model == "IC" else 0.0))
    return out


def instance_graph(inst) -> Graph:
    g = rmat(inst["scale"], seed=inst["gseed"], cache=False)
    if inst["model"] == "LT":
        g = with_weights(g, lt_weights(g, seed=inst["gseed"] + 100))
    return g
