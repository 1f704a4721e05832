#!/usr/bin/env python
"""Benchmark: memory-efficient IMM on one MI355X, one JSON line.

Default (--workload all): the headline is the largest configuration that fits one
GPU, the Chung-Lu digraph shaped like twitter7 (41.7M vertices, ~1.44B edges,
exponent 2.2, weighted cascade) with Huffman + density-gated hot-bitmap stores.
A step is one complete IMM query on it (estimation rounds of sampling, encoding
and greedy selection, then the final round), drawn from the serving stream
(k ~ U{10..200}, eps in {.5, .2}, l = 1, seed 1000 + q); --warmup queries run
untimed, then --steps queries are timed back to back with the graph resident in
HBM.  value = final RR sets of the timed queries / their time.  The same line
carries the serving loop at 0.5/0.8/1.0x the measured service rate (p50/p99,
served == alone), the roofline of the dominant kernel over a profiled second
pass of the timed queries (HBM fraction beside the Philox ALU fraction), peak
device bytes, the
oracle on the host's cores (a bounded sample; core count and CPU model), and
records of the other configurations measured in the same run:

  c2  R-MAT scale 20, IC weighted cascade, eps=.5, l=1, k=50, hot bitmap (top
      1% from a 10% warm-up; also with the 1/32 density gate);
  c3  R-MAT scale 23, LT, eps=.13, k=100, Huffman (5% warm-up);
  c4  256 R-MAT instances of scale U{12..18}, IC-WC + hot bitmap and LT +
      Huffman alternating, k ~ U{5..100}, eps in {.5, .3}: batched vs plain;
  flat  G(65536, 2^20) with IC p = 0.1 on every edge (a flat-head store), eps=.5,
      k=50, encoding chosen by Alg. 1 (Bitmax here), and the equal-memory
      comparison: the same IMM on plain ids capped at the compressed store's
      device bytes, the rest spilled to pinned host memory.

--workload c2|c3|c4|c5|flat runs one configuration as the main line.
--philox-probe measures the Philox call rate of the samplers' RNG against the
ALU peak derived from unit counts.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RR sets/s and IMM end-to-end s (batched vs plain, same GPU); compressed B/RR"

WORKLOADS = {
    "all": dict(name="imm_chunglu41.7M_1.44Bedges_icwc_huffman-hotbitmap_serving-stream", cfg="c5"),
    "c2": dict(name="imm_ic_wc_rmat20_eps0.5_k50_hotbitmap", cfg="c2"),
    "c3": dict(name="imm_lt_rmat23_eps0.13_k100_huffman", cfg="c3"),
    "flat": dict(name="imm_flathead_er65536_m1M_ic_p0.1_eps0.5_k50_auto", cfg="flat"),
    "c4": dict(name="imm_batch256_rmat12-18_icwc-hotbitmap_lt-huffman", cfg="c4"),
    "c5": dict(name="serve_chunglu41.7M_1.44Bedges_icwc_huffman-hotbitmap_poisson", cfg="c5"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
CUS, SIMDS, LANES, CLOCK_GHZ = 256, 4, 16, 2.4
# One Philox4x32-10 call as the kernels compile it: 10 rounds x (2 v_mad_u64_u32 + 4 v_xor_b32; the
# key schedule is scalar) = 60 VALU instructions, each one lane slot per lane (`--philox-probe`
# measures the call rate of the same device function over the whole chip).
PHILOX_SLOTS = 60.0
PHILOX_PEAK_G = CUS * SIMDS * LANES * CLOCK_GHZ / PHILOX_SLOTS  # G calls/s
SAMPLER_KERNELS = ("ic_sample_wave", "ic_sample_block", "ic_sample_block_xl", "ic_sample_bitmap", "lt_sample_lane",
                   "lt_sample_wave", "lt_sample_block", "sample_huge")
SELECT_KERNELS = ("argmax", "find_raw", "find_huff", "apply", "dec_hot", "dec_arr")
HOST_THREADS_CAP = 16  # the GPU machine's CPU share per GPU


def kernel_rates(kstats):
    """Algorithmic GB/s and its fraction of the HBM peak for every profiled kernel (average over
    its launches), with the Philox rate of the samplers."""
    out = []
    for r in sorted(kstats, key=lambda r: -r["total_ms"]):
        if r["total_ms"] <= 0:
            continue
        gbs = r["alg_bytes"] / (r["total_ms"] * 1e-3) / 1e9
        e = {"name": r["name"], "launches": r["launches"], "ms": round(r["total_ms"], 3),
             "alg_gbs": round(gbs, 2), "hbm_frac": round(gbs / HBM_PEAK_GBS, 5)}
        if r["alg_ops"] > 0:
            e["gphilox_s"] = round(r["alg_ops"] / (r["total_ms"] * 1e-3) / 1e9, 2)
            e["alu_frac"] = round(e["gphilox_s"] / PHILOX_PEAK_G, 4)
        out.append(e)
    return out


def roofline(kstats, model, prob, workload):
    """Roofline of the kernel with the largest total time in one profiled step: IC samplers against
    the Philox ALU peak (derived from unit counts and clock), everything else against HBM; the HBM
    fraction of the algorithmic bytes is given in both cases."""
    k = max(kstats, key=lambda r: r["total_ms"])
    avg_ms = k["total_ms"] / max(k["launches"], 1)
    per_launch_bytes = k["alg_bytes"] / max(k["launches"], 1)
    per_launch_ops = k["alg_ops"] / max(k["launches"], 1)
    hbm_gbs = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    if k["name"] in SAMPLER_KERNELS and model == "IC":
        # IC sampling does one Philox call per four in-edges of every expanded vertex and moves few
        # bytes: the integer ALU bounds it
        achieved = per_launch_ops / (avg_ms * 1e-3) / 1e9
        out = {"bound": "alu", "achieved": achieved, "peak": PHILOX_PEAK_G, "unit": "Gphilox/s"}
    else:
        out = {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["hbm_achieved_gbs"] = hbm_gbs
    out["hbm_frac"] = hbm_gbs / HBM_PEAK_GBS
    out["traffic"] = counters_for(k["name"], workload, "traffic")
    out["l2_hit_rate"] = counters_for(k["name"], workload, "l2_hit")
    out["kernel"] = k["name"]
    out["launches_per_step"] = k["launches"]
    out["avg_launch_ms"] = avg_ms
    out["alg_bytes_per_launch"] = per_launch_bytes
    out["alg_ops_per_launch"] = per_launch_ops
    return out


def csrc_digest():
    import hashlib

    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_2208_00613_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


# hbm_profile names -> the HIP kernels behind them (regular expressions over the symbol after
# "hbm::", matching the plain and grouped forms; the LDS tiers' three capacities are told apart
# by their template arguments)
PROFILE_KERNELS = {
    "ic_sample_wave": r"k_ic_t1(_g)?\b", "ic_sample_block": r"k_big_lds(_g)?<\d+, 2048,",
    "ic_sample_block_xl": r"k_big_lds(_g)?<\d+, 8192,", "ic_sample_block_s": r"k_big_lds(_g)?<\d+, 1024,",
    "ic_sample_bitmap": r"k_big(_g)?\b",
    "lt_sample_lane": r"k_lt_t1(_g)?\b", "lt_sample_wave": r"k_lt_wave(_g)?\b", "lt_sample_block": r"k_big(_g)?\b",
    "sample_huge": r"k_big(_g)?\b",
}
for _k in ("hist_add", "cold_count", "split", "huff_bits", "huff_write", "argmax", "find_raw", "find_huff", "apply",
           "dec_hot", "dec_arr"):
    PROFILE_KERNELS[_k] = r"k_" + _k + r"(_g)?\b"
COPY_BYTES = 1 << 30  # the reference copy kernel of the traffic probe moves 1 GiB each way
PROBE_FLAGS = {"c5": " --warmup 5 --steps 4"}  # the counter runs' queries: the first four timed ones
C5_BLOCK_ALONE, C5_BLOCK_SERVING = 1 << 18, 1 << 16  # sets per sampling block on the Chung-Lu graph


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"counters_{'c5' if workload == 'all' else workload}.json")


def c5_context(P, torch, want_host=False):
    """The served Chung-Lu graph, generated on the GPU and loaded into a context (encoding set)."""
    from synth import graphs as G

    c = G.C5
    t0 = time.time()
    rp, dst = G.chung_lu_csr(c["n"], c["avg_deg"], c["gamma"], c["gseed"], c["max_deg"], device="cuda")
    torch.cuda.synchronize()
    m = int(dst.numel())
    log(f"[bench] Chung-Lu n={c['n']} m={m} generated on the GPU ({time.time() - t0:.1f}s)")
    ctx = P.Context(0)
    t0 = time.time()
    ctx.hbm_load_graph(c["n"], rp, dst, None, "IC", "WC")
    log(f"[bench] Chung-Lu graph loaded ({time.time() - t0:.1f}s)")
    host = (rp.cpu().numpy(), dst.cpu().numpy()) if want_host else None
    del rp, dst
    torch.cuda.empty_cache()
    ctx.hbm_set_encoding(c["enc"], c["warmup"], c["hot"])
    ctx.hbm_set_hot_density(c["hot_density"])
    return ctx, c, m, host


def traffic_probe(args):
    """The workload of the counter runs: one IMM step of the chosen workload (for the default line:
    the timed queries of the Chung-Lu stream), then a plain 1 GiB device copy whose counter
    readings calibrate FETCH_SIZE and WRITE_SIZE."""
    import torch

    import paper_2208_00613_amd as P
    from synth import graphs as G

    if args.workload in ("all", "c5"):
        ctx, c, _, _ = c5_context(P, torch)
        ctx.hbm_set_tuning("BLOCK_SETS", C5_BLOCK_ALONE)
        # the timed queries of the default line (a few of them: counters serialize every dispatch)
        for q in G.serving_queries(args.warmup + args.steps, seed=c["gseed"], rate=1.0)[args.warmup:]:
            ctx.hbm_imm(q["k"], q["eps"], q["l"], q["seed"])
            log(f"[traffic] query {q['q']} done")
    else:
        c = G.CONFIGS[WORKLOADS[args.workload]["cfg"]]
        g = G.config_graph(WORKLOADS[args.workload]["cfg"])
        ctx = P.Context(0)
        ctx.load_synth(g, model=c["model"], prob=c["prob"])
        ctx.hbm_set_encoding(c["enc"], c.get("warmup", 0.1), c.get("hot", 0.01))
        ctx.hbm_imm(c["k"], c["eps"], c["l"], c["seed"])
    torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("[traffic] probe done")
    ctx.close()


def counters_summarize(fetch_csv, write_csv, l2_csv, workload, out_path=None):
    """Per-kernel averages from rocprofv3 --pmc runs of the traffic probe: HBM bytes per launch
    (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by the reading of the 1 GiB copy)
    and the L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS).  Writes profiles/counters_<workload>.json."""
    import csv
    import re

    def per_kernel(path, counter, scale=1.0):
        """Kernel name -> values in dispatch order, and the last three dispatches (the probe's
        closing copies) as (name, value)."""
        import gzip

        acc, rows = {}, []
        if not path:
            return acc, rows
        f = gzip.open(path, "rt") if path.endswith(".gz") else open(path)
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * scale))
        rows.sort()
        for _, k, v in rows:
            acc.setdefault(k, []).append(v)
        return acc, [(k, v) for _, k, v in rows[-3:]]

    (fetch, f_last), (write, w_last) = per_kernel(fetch_csv, "FETCH_SIZE", 1024.0), per_kernel(write_csv, "WRITE_SIZE", 1024.0)
    (hit, _), (miss, _) = per_kernel(l2_csv, "TCC_HIT_sum"), per_kernel(l2_csv, "TCC_MISS_sum")
    # the probe ends with three 1 GiB device copies: its last three dispatches calibrate the counters
    names = {k for k, _ in f_last} | {k for k, _ in w_last}
    if len(f_last) < 3 or len(names) != 1 or "hbm::" in next(iter(names)):
        raise SystemExit("the counter run does not end with the probe's three copies")
    ck = next(iter(names))
    f_scale = COPY_BYTES / float(np.median([v for _, v in f_last]))
    w_scale = COPY_BYTES / float(np.median([v for _, v in w_last])) if w_last else 1.0
    traffic, l2 = {}, {}
    mean = lambda v: sum(v) / len(v)
    for prof, sym in PROFILE_KERNELS.items():
        pat = re.compile(r"hbm::" + sym)
        fs = [x for k, v in fetch.items() if pat.search(k) for x in v]
        ws = [x for k, v in write.items() if pat.search(k) for x in v]
        if fs:
            traffic[prof] = mean(fs) * f_scale + (mean(ws) * w_scale if ws else 0.0)
        hs = sum(x for k, v in hit.items() if pat.search(k) for x in v)
        ms = sum(x for k, v in miss.items() if pat.search(k) for x in v)
        if hs + ms > 0:
            l2[prof] = hs / (hs + ms)
    wl = "c5" if workload == "all" else workload
    probe = PROBE_FLAGS.get(wl, "")
    cmds = [f"cd /tmp && rocprofv3 --pmc {ctr} -f csv -d $GRAFT_REPO_ROOT/gpurun_out/pmc_{tag} -o {tag} -- "
            f"python $GRAFT_REPO_ROOT/bench.py --traffic-probe --workload {wl}{probe}"
            for ctr, tag in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"), ("TCC_HIT_sum TCC_MISS_sum", "l2"))]
    cmds.append(f"python bench.py --workload {wl} --counters-summarize gpurun_out/pmc_fetch/fetch_counter_collection.csv.gz "
                "gpurun_out/pmc_write/write_counter_collection.csv.gz gpurun_out/pmc_l2/l2_counter_collection.csv.gz")
    what = ("queries 5..8 of the serving stream (the first four timed queries of the default line)" if wl == "c5"
            else "one IMM step")
    out = {"commands": cmds, "workload": WORKLOADS[wl]["name"] + ", " + what, "workload_key": wl,
           "csrc_digest": csrc_digest(), "copy_kernel": ck[:80], "fetch_scale": f_scale, "write_scale": w_scale,
           "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)", "traffic": traffic,
           "l2_hit_unit": "TCC_HIT / (TCC_HIT + TCC_MISS) over the kernel's launches", "l2_hit": l2}
    json.dump(out, open(out_path or counters_path(wl), "w"), indent=1)
    print(json.dumps(out))


def counters_for(kernel, workload, what):
    """A counter figure for a kernel, if taken on the current kernels and on this workload."""
    path = counters_path(workload)
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("csrc_digest") != csrc_digest():
        return None
    return t.get(what, {}).get(kernel)


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity": avail, "cpu_model": model,
            "threads": max(1, min(HOST_THREADS_CAP, avail))}


def oracle_sample_rate(og, seed, budget_s, threads, chunk):
    """RR sets per second of the oracle sampling shards of one index range on `threads` threads
    (each shard a store of its own; the C calls release the GIL)."""
    import threading

    import oracle

    nxt = [0]
    lock = threading.Lock()
    stores = []
    scratch = [oracle.Scratch(og.n) for _ in range(threads)]  # one per thread: the graph's own is not shared
    t0 = time.perf_counter()

    def work(sc):
        st = oracle.Store()
        stores.append(st)
        while True:
            with lock:
                if time.perf_counter() - t0 > budget_s:
                    return
                j0 = nxt[0]
                nxt[0] += chunk
            st.append_range(og, seed, j0, j0 + chunk, sc)

    ts = [threading.Thread(target=work, args=(sc,)) for sc in scratch]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    secs = time.perf_counter() - t0
    return nxt[0] / secs, nxt[0], secs


def cpu_baseline(og, n, seed, k, t_graph, label, budget_s=8.0, chunk=500):
    """The oracle as it stands on a bounded sample of the same RR-set stream: one core sampling a
    prefix then running its greedy over it, and all host cores (up to the GPU machine's share)
    sampling shards of the index range."""
    import oracle

    hi = host_info()
    st = oracle.Store()
    theta = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s:
        theta += chunk
        st.extend(og, seed, theta)
    t_sample = time.perf_counter() - t1
    t2 = time.perf_counter()
    oracle.greedy(st, n, k)
    t_select = time.perf_counter() - t2
    del st
    rate, sets, secs = oracle_sample_rate(og, seed, budget_s, hi["threads"], chunk)
    return {"value": rate, "unit": "RR sets/s", "cores": hi["threads"], "kind": "oracle",
            "sample": f"{label}: RR sets 0..{sets - 1} of the seed-{seed} stream sampled in shards of {chunk} on "
                      f"{hi['threads']} threads ({secs:.1f}s); graph transpose ({t_graph:.1f}s) excluded",
            "one_core": {"value": theta / (t_sample + t_select), "unit": "RR sets/s",
                         "sample": f"RR sets 0..{theta - 1} sampled, then greedy k={k} on them",
                         "seconds": t_sample + t_select},
            "nproc": hi["nproc"], "affinity": hi["affinity"], "cpu_model": hi["cpu_model"]}


def oracle_graph(n, row_ptr, dst, w, model, prob):
    import oracle

    oracle.build()
    t0 = time.perf_counter()
    og = oracle.Graph(n, row_ptr, dst, w, model=model, prob=prob)
    return og, time.perf_counter() - t0


def _instance_graph(inst):
    from synth import graphs as G

    return G.instance_graph(inst)


def _config_graph(name):
    from synth import graphs as G

    return G.config_graph(name)


def start_host_work(pool, names, batched_count):
    """Graph generation in a process pool (forked before anything touches the GPU)."""
    from synth import graphs as G

    futs = {nm: pool.submit(_config_graph, nm) for nm in names}
    insts = G.batched_instances(count=batched_count) if batched_count else None
    bfuts = [pool.submit(_instance_graph, i) for i in insts] if insts else None
    return futs, insts, bfuts


def batched_setup(P, insts, graphs):
    """Load every instance graph into its own context (resident in HBM) with its encoding."""
    ctxs = []
    for inst, g in zip(insts, graphs):
        c = P.Context(0)
        c.load_synth(g, inst["model"], inst["prob"])
        c.hbm_set_encoding(inst["enc"], inst["warmup"], inst["hot"] or 0.01)
        ctxs.append(c)
    return ctxs


def batched_vs_plain(P, torch, ctxs, insts, reps=1):
    """Whole-workload seconds of hbm_imm_batch vs one hbm_imm per instance, same GPU, same
    queries; the results must agree instance by instance."""
    qs = [(i["k"], i["eps"], i["l"], i["seed"]) for i in insts]
    # launch shapes from the autotuner (applied to every context: both paths use them)
    tuning, _ = P.imm_autotune(ctxs, qs)
    log(f"[bench] autotuned: {tuning}")
    P.imm_batch(ctxs, qs)  # warm-up: allocations of both paths
    for c, q in zip(ctxs, qs):
        c.hbm_imm(*q)
    tb, tp = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = P.imm_batch(ctxs, qs)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        plain = [c.hbm_imm(*q) for c, q in zip(ctxs, qs)]
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
    same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(out, plain))
    sets = sum(o[2]["nsets_final"] for o in out)
    store = sum(o[2]["store"]["store_bytes"] for o in out)
    raw = sum(4 * o[2]["store"]["members"] + 8 * (o[2]["nsets_final"] + 1) for o in out)
    peak = sum(c.hbm_get_memory()[1] for c in ctxs)
    return dict(instances=len(ctxs), tuning=tuning, batched_s=min(tb), plain_s=min(tp), speedup=min(tp) / min(tb),
                identical_results=bool(same), rr_sets=sets, bytes_per_rr=store / max(sets, 1),
                raw_bytes_per_rr=raw / max(sets, 1), peak_device_bytes=peak), out


def cpu_baseline_batched(insts, graphs, budget_s=8.0):
    """The oracle's full IMM, instance after instance in workload order, until the time budget."""
    import oracle

    oracle.build()
    t0 = time.perf_counter()
    sets, done = 0, 0
    for inst, g in zip(insts, graphs):
        og = oracle.Graph(g.n, g.row_ptr, g.dst, g.w if inst["prob"] == "EDGE" else None, model=inst["model"],
                          prob=inst["prob"])
        _, _, st, _ = oracle.imm(og, inst["k"], inst["eps"], inst["l"], inst["seed"])
        sets += st["nsets_final"]
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    secs = time.perf_counter() - t0
    hi = host_info()
    return {"value": sets / secs, "unit": "RR sets/s", "cores": 1, "kind": "oracle",
            "sample": f"full oracle IMM of the first {done} of {len(insts)} instances ({sets} RR sets, graph "
                      f"transposes included)", "seconds": secs, "nproc": hi["nproc"], "cpu_model": hi["cpu_model"]}


def main_c4(args, P, torch, insts, graphs):
    wl = WORKLOADS["c4"]
    ctxs = batched_setup(P, insts, graphs)
    cmp_, out = batched_vs_plain(P, torch, ctxs, insts, reps=max(1, args.steps))
    qs = [(i["k"], i["eps"], i["l"], i["seed"]) for i in insts]
    ctxs[0].hbm_profile(True)
    P.imm_batch(ctxs, qs)
    kstats = ctxs[0].hbm_profile_read()
    ctxs[0].hbm_profile(False)
    ms = cmp_["batched_s"] * 1e3
    res = {
        "metric": METRIC, "value": cmp_["rr_sets"] / cmp_["batched_s"], "unit": "RR sets/s", "n_gpus": 1,
        "steps": max(1, args.steps), "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded R-MAT instances; no public dataset)",
        "config": {"workload": wl["name"], "instances": len(insts), "scales": "U{12..18}", "k": "U{5..100}",
                   "eps": [0.5, 0.3]},
        "imm_s": cmp_["batched_s"], "batched_vs_plain": cmp_,
        "phase_ms": {"sample_encode": out[0][2]["t_sample_ms"], "select": out[0][2]["t_select_ms"]},
        "roofline": roofline(kstats, "IC", "WC", args.workload),
        "kernels": kernel_rates(kstats)[:10],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_batched(insts, graphs)
    print(json.dumps(res), flush=True)
    for c in ctxs:
        c.close()


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def serve_level(P, ctx, queries, budget, max_active):
    """Replay one Poisson arrival stream against a fresh server; returns per-query results."""
    srv = P.Server(ctx, store_budget=budget, max_active=max_active)
    t0 = time.perf_counter()
    tickets = []
    for q in queries:
        while time.perf_counter() - t0 < q["t"]:
            time.sleep(min(0.005, max(0.0, q["t"] - (time.perf_counter() - t0))))
        tickets.append(srv.hbm_server_submit(q["k"], q["eps"], q["l"], q["seed"]))
    res = [srv.hbm_server_poll(t, wait=True) for t in tickets]
    st = srv.hbm_server_get_stats()
    srv.close()
    return res, st


def serving_levels(P, ctx, c, alone, svc, nq, loads):
    """Poisson arrivals of the first nq stream queries at fractions of the service rate; each
    served answer against the same query alone."""
    from synth import graphs as G

    levels, identical = {}, True
    for load in loads:
        qs = G.serving_queries(nq, seed=c["gseed"], rate=load / svc)
        res, st = serve_level(P, ctx, qs, c["budget"], 16)
        lat = [r["t_done_ms"] - r["t_submit_ms"] for r in res]
        span = (max(r["t_done_ms"] for r in res) - min(r["t_submit_ms"] for r in res)) / 1e3
        ok = all(r["status"] == "OK" for r in res)
        same = ok and all(np.array_equal(r["seeds"], alone[q["q"]][0]) and np.array_equal(r["gains"], alone[q["q"]][1])
                          for r, q in zip(res, qs))
        identical &= same
        sets = sum(r["stats"]["nsets_final"] for r in res if r["status"] == "OK")
        levels[str(load)] = dict(rate_qps=load / svc, queries=nq, p50_ms=pct(lat, 50), p99_ms=pct(lat, 99),
                                 mean_ms=float(np.mean(lat)), makespan_s=span, queries_per_s=nq / span,
                                 rr_sets_per_s=sets / span, served_equals_alone=bool(same),
                                 peak_active=st["peak_active"], preemptions=st["preemptions"],
                                 peak_store_bytes=st["peak_store_bytes"], steps=st["steps"])
        log(f"[bench] load {load}: p50 {levels[str(load)]['p50_ms']:.0f} ms p99 {levels[str(load)]['p99_ms']:.0f} ms "
            f"{nq / span:.2f} q/s peak_active {st['peak_active']} same={same}")
    return levels, identical


def c5_record(args, P, torch, with_host):
    """The headline: IMM queries of the serving stream on the Chung-Lu graph, timed back to back
    alone; then a profiled pass over the same queries, peak bytes, the serving loop at each load."""
    from synth import graphs as G

    ctx, c, m, host = c5_context(P, torch, want_host=with_host)
    # queries alone run in blocks of 2^18 sets (fewer tier launches and host round trips); the
    # serving loop below uses 2^16, so arrivals join within a block's time
    ctx.hbm_set_tuning("BLOCK_SETS", C5_BLOCK_ALONE)
    W, K = args.warmup, args.steps
    nq = max(args.queries, W + K)
    stream = G.serving_queries(nq, seed=c["gseed"], rate=1.0)
    alone = {}
    for q in stream[:W]:
        alone[q["q"]] = ctx.hbm_imm(q["k"], q["eps"], q["l"], q["seed"])
    ctx.hbm_get_memory(reset_peak=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in stream[W:W + K]:
        alone[q["q"]] = ctx.hbm_imm(q["k"], q["eps"], q["l"], q["seed"])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    _, peak = ctx.hbm_get_memory()
    timed = [alone[q["q"]][2] for q in stream[W:W + K]]
    sets = sum(st["nsets_final"] for st in timed)
    log(f"[bench] {K} timed queries alone: {secs:.3f}s, {sets} RR sets")
    t_alone = []
    for q in stream[W + K:]:
        t1 = time.perf_counter()
        alone[q["q"]] = ctx.hbm_imm(q["k"], q["eps"], q["l"], q["seed"])
        t_alone.append(time.perf_counter() - t1)
    svc = (secs + sum(t_alone)) / (K + len(t_alone))
    # one profiled pass over the same K queries: per-kernel HIP-event times and algorithmic work
    ctx.hbm_profile(True)
    for q in stream[W:W + K]:
        ctx.hbm_imm(q["k"], q["eps"], q["l"], q["seed"])
    kstats = ctx.hbm_profile_read()
    ctx.hbm_profile(False)
    # implicit roots, then array rows for the sparse hot vertices, on the first timed query:
    # B/RR beside the plain store's
    q0 = stream[W]
    st_0 = alone[q0["q"]][2]
    variants = {}
    for name, setter in (("implicit_roots", ctx.hbm_set_implicit_roots), ("row_containers", ctx.hbm_set_row_containers)):
        setter(True)
        s_i, g_i, st_i = ctx.hbm_imm(q0["k"], q0["eps"], q0["l"], q0["seed"])
        setter(False)
        variants[name] = {
            "query": {"k": q0["k"], "eps": q0["eps"], "seed": q0["seed"]},
            "bytes_per_rr": st_i["store"]["store_bytes"] / st_i["nsets_final"],
            "plain_bytes_per_rr": st_0["store"]["store_bytes"] / st_0["nsets_final"],
            "narray": st_i["store"]["narray"], "nhot": st_i["store"]["nhot"],
            "same_seeds": bool(np.array_equal(s_i, alone[q0["q"]][0]) and np.array_equal(g_i, alone[q0["q"]][1]))}
    ctx.hbm_set_tuning("BLOCK_SETS", C5_BLOCK_SERVING)
    levels, identical = serving_levels(P, ctx, c, alone, svc, args.queries, args.loads)
    stores = [st["store"] for st in timed]
    rec = {
        "value": sets / secs, "ms_per_step": secs * 1e3 / K, "imm_s_mean": secs / K,
        "config": {"workload": WORKLOADS["all"]["name"], "n": c["n"], "m": m, "gamma": c["gamma"], "model": "IC",
                   "prob": "WC", "k": "U{10..200}", "eps": [0.5, 0.2], "l": 1.0, "timed_queries": K,
                   "warmup_queries": W, "query_seeds": f"1000+q, q = {W}..{W + K - 1}", "encoding": c["enc"],
                   "hot_frac": c["hot"], "hot_min_density": c["hot_density"], "warmup_frac": c["warmup"],
                   "store_budget_bytes": c["budget"], "block_sets_alone": C5_BLOCK_ALONE,
                   "block_sets_serving": C5_BLOCK_SERVING},
        "rr_sets": sets, "theta_final_range": [min(st["theta_final"] for st in timed),
                                               max(st["theta_final"] for st in timed)],
        "bytes_per_rr": sum(s_["store_bytes"] for s_ in stores) / max(sets, 1),
        "raw_bytes_per_rr": sum(4 * s_["members"] + 8 * (s_["nsets"] + 1) for s_ in stores) / max(sets, 1),
        "payload_bits_per_occurrence": sum(s_["payload_bits"] for s_ in stores) / max(
            sum(s_["members"] for s_ in stores), 1),
        "peak_device_bytes": peak,
        "phase_ms_mean": {"sample_encode": float(np.mean([st["t_sample_ms"] for st in timed])),
                          "select": float(np.mean([st["t_select_ms"] for st in timed])),
                          "model_of_which": float(np.mean([st["t_encode_ms"] for st in timed]))},
        "profiled": f"a second pass over the {K} timed queries with per-launch HIP events",
        "roofline": roofline(kstats, "IC", "WC", "all"),
        "kernels": kernel_rates(kstats)[:12],
        "serving": {"levels": levels, "served_equals_alone": bool(identical), "mean_service_s": svc},
        **variants,
    }
    return ctx, c, rec, host


def variant_leg(torch, ctx, c, seeds, gains, rec, setter):
    """The same IMM with one store option on (implicit roots: each set's root regenerated from
    Philox, not stored; row containers: array rows for the sparse hot vertices): B/RR and time
    beside the plain store's, and the seeds (which must not change)."""
    k, eps, l, seed = c["k"], c["eps"], c["l"], c["seed"]
    setter(True)
    ctx.hbm_imm(k, eps, l, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s2, g2, st2 = ctx.hbm_imm(k, eps, l, seed)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    setter(False)
    return {"bytes_per_rr": st2["store"]["store_bytes"] / max(st2["nsets_final"], 1),
            "plain_bytes_per_rr": rec["bytes_per_rr"], "imm_s": t, "plain_imm_s": rec["imm_s"],
            "narray": st2["store"]["narray"], "nhot": st2["store"]["nhot"],
            "same_seeds": bool(np.array_equal(s2, seeds) and np.array_equal(g2, gains))}


def imm_record(P, torch, g, c, wl_key, steps, warmup, density_gate=False, equal_memory=False):
    """Full IMM on one R-MAT configuration: timed steps, one profiled step, B/RR, peak bytes."""
    ctx = P.Context(0)
    ctx.load_synth(g, model=c["model"], prob=c["prob"])
    ctx.hbm_set_encoding(c["enc"], c.get("warmup", 0.1), c.get("hot", 0.01))
    torch.cuda.synchronize()
    k, eps, l, seed = c["k"], c["eps"], c["l"], c["seed"]
    for i in range(warmup):
        _, _, st = ctx.hbm_imm(k, eps, l, seed)
        log(f"[bench] {wl_key} warmup {i}: {st['t_total_ms']:.1f} ms, theta={st['nsets_final']}")
    ctx.hbm_get_memory(reset_peak=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seeds, gains, st = ctx.hbm_imm(k, eps, l, seed)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    _, peak = ctx.hbm_get_memory()
    nsets = st["nsets_final"]
    store = st["store"]
    rec = {
        "value": nsets / (ms / 1e3), "ms_per_step": ms, "imm_s": ms / 1e3, "steps": steps, "warmup": warmup,
        "config": {"workload": WORKLOADS[wl_key]["name"], "n": g.n, "m": g.m, "model": c["model"], "prob": c["prob"],
                   "k": k, "eps": eps, "l": l, "encoding": c["enc"], "seed": seed},
        "theta_final": st["theta_final"], "nsets": nsets, "rounds": st["rounds"], "coverage": st["coverage"],
        "influence": st["influence"],
        "bytes_per_rr": store["store_bytes"] / max(nsets, 1),
        "raw_bytes_per_rr": (4 * store["members"] + 8 * (nsets + 1)) / max(nsets, 1),
        "skewness": store["skewness"], "density": store["density"], "encoding_used": store["encoding"],
        "peak_device_bytes": peak,
        "phase_ms": {"sample_encode": st["t_sample_ms"], "select": st["t_select_ms"],
                     "model_of_which": st["t_encode_ms"]},
    }
    ctx.hbm_profile(True)
    ctx.hbm_imm(k, eps, l, seed)
    kstats = ctx.hbm_profile_read()
    ctx.hbm_profile(False)
    rec["roofline"] = roofline(kstats, c["model"], c["prob"], wl_key)
    rec["kernels"] = kernel_rates(kstats)[:10]
    if density_gate:
        # the same IMM with the hot set gated at density 1/32 (a row only where it is the smaller form)
        ctx.hbm_set_hot_density(1.0 / 32)
        ctx.hbm_imm(k, eps, l, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s2, g2, st2 = ctx.hbm_imm(k, eps, l, seed)
        t_g = time.perf_counter() - t0
        rec["density_gate_1_32"] = {
            "bytes_per_rr": st2["store"]["store_bytes"] / max(st2["nsets_final"], 1), "imm_s": t_g,
            "nhot": st2["store"]["nhot"], "same_seeds": bool(np.array_equal(s2, seeds) and np.array_equal(g2, gains))}
        ctx.hbm_set_hot_density(0.0)
    if equal_memory:
        rec["equal_memory"] = equal_memory_leg(P, torch, ctx, c, seeds, gains, rec)
    elif c["enc"] != "BITMAX":
        rec["implicit_roots"] = variant_leg(torch, ctx, c, seeds, gains, rec, ctx.hbm_set_implicit_roots)
        if c["enc"] in ("HOT_BITMAP", "HUFFMAN_HOT_BITMAP"):
            rec["row_containers"] = variant_leg(torch, ctx, c, seeds, gains, rec, ctx.hbm_set_row_containers)
    ctx.close()
    return rec


def equal_memory_leg(P, torch, ctx, c, seeds, gains, rec):
    """The Evaluation section's equal-memory comparison on one GPU: the same IMM with a plain-id
    store that may keep on the device only as many bytes as the compressed store took; the rest
    of its ids spill to pinned host memory, read over the bus by the selection kernels."""
    k, eps, l, seed = c["k"], c["eps"], c["l"], c["seed"]
    cap = int(rec["bytes_per_rr"] * rec["nsets"])
    ctx.hbm_set_encoding("NONE")
    ctx.hbm_set_spill(cap)
    ctx.hbm_imm(k, eps, l, seed)  # warm-up (allocations, host part)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s2, g2, st2 = ctx.hbm_imm(k, eps, l, seed)
    torch.cuda.synchronize()
    t_spill = time.perf_counter() - t0
    raw_bytes = st2["store"]["store_bytes"]
    ctx.hbm_set_spill(0)
    ctx.hbm_imm(k, eps, l, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s3, g3, st3 = ctx.hbm_imm(k, eps, l, seed)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    ctx.hbm_set_encoding(c["enc"], c.get("warmup", 0.1), c.get("hot", 0.01))
    return {"compressed_store_bytes": cap, "compressed_imm_s": rec["imm_s"],
            "compressed_encoding": rec.get("encoding_used"),
            "plain_store_bytes": raw_bytes, "plain_device_bytes_cap": cap,
            "plain_spilled_bytes": max(0, raw_bytes - cap), "plain_spilled_imm_s": t_spill,
            "plain_all_on_device_imm_s": t_dev,
            "speedup_compressed_vs_spilled": t_spill / rec["imm_s"],
            "same_seeds": bool(np.array_equal(s2, seeds) and np.array_equal(g2, gains)
                               and np.array_equal(s3, seeds) and np.array_equal(g3, gains))}


def philox_probe(P, torch):
    """The samplers' Philox device function over the whole chip, against the ALU peak."""
    ctx = P.Context(0)
    blocks, calls = CUS * 8, 4096
    ctx.hbm_bench_philox(64, blocks)
    best = None
    for _ in range(5):
        ms, chk = ctx.hbm_bench_philox(calls, blocks)
        best = ms if best is None else min(best, ms)
    g = blocks * 256 * calls / (best * 1e-3) / 1e9
    ctx.close()
    return {"metric": "Philox4x32-10 calls/s", "value": g, "unit": "G calls/s", "peak": PHILOX_PEAK_G,
            "frac": g / PHILOX_PEAK_G, "blocks": blocks, "threads_per_block": 256, "calls_per_thread": calls,
            "kernel_ms": best, "checksum": chk,
            "peak_derivation": f"{CUS} CU x {SIMDS} SIMD x {LANES} lanes x {CLOCK_GHZ} GHz / {PHILOX_SLOTS:.0f} "
                               "VALU slots per call"}


def main_all(args, P, torch, pool, futs, insts, bfuts):
    """The default line: the Chung-Lu headline, with the c2, c3 and c4 records of the same run."""
    from synth import graphs as G

    ctx, c, rec, host = c5_record(args, P, torch, with_host=not args.no_cpu_baseline)
    out = {"metric": METRIC, "value": rec["value"], "unit": "RR sets/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32",
           "data": "synthetic (seeded Chung-Lu digraph shaped like twitter7, R-MAT; no public dataset)"}
    out.update({k: v for k, v in rec.items() if k not in ("value", "ms_per_step")})
    ctx.close()
    if host is not None:
        rp_h, dst_h = host
        og, t_graph = oracle_graph(c["n"], rp_h, dst_h, None, "IC", "WC")
        del rp_h, dst_h
        hq = G.serving_queries(args.warmup + 1, seed=c["gseed"], rate=1.0)[args.warmup]
        out["cpu_baseline"] = cpu_baseline(og, c["n"], hq["seed"], hq["k"], t_graph,
                                           f"Chung-Lu query k={hq['k']} eps={hq['eps']}")
        del og
        log("[bench] c5 oracle baseline done")
    others = {}
    for key, steps, warm in (("c2", 10, 2), ("c3", 3, 1), ("flat", 3, 1)):
        t0 = time.time()
        g = futs[key].result()
        log(f"[bench] graph {key} ready ({time.time() - t0:.1f}s wait)")
        cc = G.CONFIGS[key]
        others[key] = imm_record(P, torch, g, cc, key, steps, warm, density_gate=(key == "c2"),
                                 equal_memory=(key == "flat"))
        if not args.no_cpu_baseline and key != "flat":
            og, t_graph = oracle_graph(g.n, g.row_ptr, g.dst, g.w if cc["prob"] == "EDGE" else None, cc["model"],
                                       cc["prob"])
            others[key]["cpu_baseline"] = cpu_baseline(og, g.n, cc["seed"], cc["k"], t_graph, key, budget_s=5.0)
            del og
        del g
        log(f"[bench] {key}: {others[key]['ms_per_step']:.1f} ms per IMM")
    graphs = [f.result() for f in bfuts]
    pool.shutdown()
    ctxs = batched_setup(P, insts, graphs)
    others["c4"], _ = batched_vs_plain(P, torch, ctxs, insts, reps=1)
    others["c4"]["workload"] = WORKLOADS["c4"]["name"]
    for c4 in ctxs:
        c4.close()
    out["configs"] = others
    out["batched_vs_plain"] = others["c4"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="all", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="c2 line: skip the batched-vs-plain summary")
    ap.add_argument("--queries", type=int, default=64, help="serving: queries per load level")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 0.8, 1.0],
                    help="serving: arrival rates as fractions of the measured single-query service rate")
    ap.add_argument("--philox-probe", action="store_true",
                    help="measure the Philox call rate of the samplers' RNG and exit")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the workload of the counter runs (one IMM, then a 1 GiB copy) and exit")
    ap.add_argument("--counters-summarize", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "L2_CSV"),
                    help="turn three rocprofv3 --pmc counter files into profiles/counters_<workload>.json")
    args = ap.parse_args()
    if args.counters_summarize:
        return counters_summarize(*args.counters_summarize, args.workload)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU sharding is described in "
                                   "DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.traffic_probe:
        return traffic_probe(args)

    import concurrent.futures as cf

    pool = futs = insts = bfuts = None
    if args.workload == "all":
        pool = cf.ProcessPoolExecutor(8)
        futs, insts, bfuts = start_host_work(pool, ["c2", "c3", "flat"], 256)
    elif args.workload == "c4" or (args.workload == "c2" and not args.no_batched):
        pool = cf.ProcessPoolExecutor(8)
        _, insts, bfuts = start_host_work(pool, [], 256)

    import torch

    import paper_2208_00613_amd as P
    from synth import graphs as G

    if args.philox_probe:
        print(json.dumps(philox_probe(P, torch)), flush=True)
        return
    if args.workload == "all":
        return main_all(args, P, torch, pool, futs, insts, bfuts)
    if args.workload == "c4":
        graphs = [f.result() for f in bfuts]
        pool.shutdown()
        return main_c4(args, P, torch, insts, graphs)
    if args.workload == "c5":
        ctx, c, rec, host = c5_record(args, P, torch, with_host=False)
        ctx.close()
        out = {"metric": METRIC, "unit": "RR sets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
               "data": "synthetic (seeded Chung-Lu digraph; no public dataset)"}
        out.update(rec)
        print(json.dumps(out), flush=True)
        return
    wl = WORKLOADS[args.workload]
    c = G.CONFIGS[wl["cfg"]]
    t0 = time.time()
    g = G.config_graph(wl["cfg"])
    log(f"[bench] graph {g.name}: n={g.n} m={g.m} ({time.time() - t0:.1f}s)")
    rec = imm_record(P, torch, g, c, args.workload, args.steps, args.warmup, density_gate=(args.workload == "c2"),
                     equal_memory=(args.workload == "flat"))
    out = {"metric": METRIC, "unit": "RR sets/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded R-MAT; no public dataset)"}
    out.update(rec)
    if not args.no_cpu_baseline:
        og, t_graph = oracle_graph(g.n, g.row_ptr, g.dst, g.w if c["prob"] == "EDGE" else None, c["model"], c["prob"])
        out["cpu_baseline"] = cpu_baseline(og, g.n, c["seed"], c["k"], t_graph, args.workload)
    if args.workload == "c2" and not args.no_batched:
        graphs = [f.result() for f in bfuts]
        pool.shutdown()
        ctxs = batched_setup(P, insts, graphs)
        out["batched_vs_plain"], _ = batched_vs_plain(P, torch, ctxs, insts, reps=1)
        out["batched_vs_plain"]["workload"] = WORKLOADS["c4"]["name"]
        for c4 in ctxs:
            c4.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
