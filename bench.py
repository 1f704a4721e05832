#!/usr/bin/env python
"""Benchmark: full IMM on one MI355X, one JSON line.

A step is one complete IMM run (hbm_imm): estimation rounds with RR-set
sampling, hot-bitmap encoding and k-seed greedy selection each, then the final
sampling and selection.  Default workload (c2): R-MAT scale 20 (a=.57, b=.19,
c=.19, 16 * 2^20 samples, self-loops and duplicates removed), IC with weighted
cascade probabilities, eps=0.5, l=1, k=50, hot bitmap for the top 1% of
vertices by frequency in the first 10% of sets, Philox seed 42.  The graph is
loaded into HBM before timing; the timed region holds only hbm_imm calls.

value = RR sets per second of the whole IMM run (final store size / step
time).  Extra fields report IMM seconds, compressed bytes per RR set, the
roofline of the dominant kernel, the CPU oracle baseline, and (unless
--no-batched) the batched workload's whole time batched vs plain on the same
GPU: 256 R-MAT instances of scale U{12..18}, IC-WC + hot bitmap and LT +
Huffman alternating, k ~ U{5..100}, eps in {.5, .3}.

--workload c3: R-MAT scale 23 under LT, eps=.13, k=100, Huffman (5% warm-up).
--workload c4: the batched workload as the main line (value = RR sets/s of
hbm_imm_batch over all 256 instances).
--workload c5: the serving loop on a Chung-Lu digraph shaped like twitter7
(41.7M vertices, ~1.44B edges, exponent 2.2, weighted cascade): Poisson
arrivals of queries (k ~ U{10..200}, eps in {.5, .2}) at fractions of the
measured single-query service rate, 200 GB store budget; p50/p99 latency,
throughput, and each served answer against the same query run alone.
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
    "c2": dict(name="imm_ic_wc_rmat20_eps0.5_k50_hotbitmap", cfg="c2"),
    "c3": dict(name="imm_lt_rmat23_eps0.13_k100_huffman", cfg="c3"),
    "c4": dict(name="imm_batch256_rmat12-18_icwc-hotbitmap_lt-huffman", cfg="c4"),
    "c5": dict(name="serve_chunglu41.7M_1.44Bedges_icwc_huffman-hotbitmap_poisson", cfg="c5"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
CUS, SIMDS, LANES, CLOCK_GHZ = 256, 4, 16, 2.4
# One Philox4x32-10 call as the kernels compile it: 10 rounds x (2 v_mad_u64_u32 + 4 v_xor_b32; the
# key schedule is scalar) = 60 VALU instructions, each one lane slot per lane (a plain loop of calls
# measured on MI355X reaches 638 G calls/s, 97 % of the bound below).
PHILOX_SLOTS = 60.0
PHILOX_PEAK_G = CUS * SIMDS * LANES * CLOCK_GHZ / PHILOX_SLOTS  # G calls/s
SAMPLER_KERNELS = ("ic_sample_wave", "ic_sample_block", "ic_sample_block_xl", "ic_sample_bitmap", "lt_sample_lane",
                   "lt_sample_wave", "lt_sample_block", "sample_huge")


def roofline(kstats, model, prob, workload):
    """Roofline of the kernel with the largest total time in one profiled step."""
    k = max(kstats, key=lambda r: r["total_ms"])
    avg_ms = k["total_ms"] / max(k["launches"], 1)
    per_launch_bytes = k["alg_bytes"] / max(k["launches"], 1)
    per_launch_ops = k["alg_ops"] / max(k["launches"], 1)
    if k["name"] in SAMPLER_KERNELS and model == "IC":
        # IC sampling does one Philox call per four in-edges of every expanded vertex and moves few
        # bytes: the integer ALU bounds it (peak derived from unit counts and clock)
        achieved = per_launch_ops / (avg_ms * 1e-3) / 1e9
        out = {"bound": "alu", "achieved": achieved, "peak": PHILOX_PEAK_G, "unit": "Gphilox/s"}
    else:
        achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = traffic_for(k["name"], workload)
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
# "hbm::", matching the plain and grouped forms; the LDS tier's two capacities are told apart by
# their template arguments)
PROFILE_KERNELS = {
    "ic_sample_wave": r"k_ic_t1(_g)?\b", "ic_sample_block": r"k_big_lds(_g)?<\d+, 2048,",
    "ic_sample_block_xl": r"k_big_lds(_g)?<\d+, 8192,", "ic_sample_bitmap": r"k_big(_g)?\b",
    "lt_sample_lane": r"k_lt_t1(_g)?\b", "lt_sample_wave": r"k_lt_wave(_g)?\b", "lt_sample_block": r"k_big(_g)?\b",
    "sample_huge": r"k_big(_g)?\b",
}
for _k in ("hist_add", "cold_count", "split", "huff_bits", "huff_write", "argmax", "find_raw", "find_huff", "apply",
           "dec_big", "dec_hot"):
    PROFILE_KERNELS[_k] = r"k_" + _k + r"(_g)?\b"
COPY_BYTES = 1 << 30  # the reference copy kernel of the traffic probe moves 1 GiB each way


def traffic_probe(args):
    """The workload of the counter runs: one profiled-size IMM step of the chosen workload, then
    a plain 1 GiB device copy whose counter readings calibrate FETCH_SIZE and WRITE_SIZE."""
    import torch

    import paper_2208_00613_amd as P
    from synth import graphs as G

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


def traffic_summarize(fetch_csv, write_csv, out_path, workload):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per kernel from two rocprofv3 --pmc runs,
    each scaled by the reading of the 1 GiB copy; writes HBM bytes per launch per profile name."""
    import csv
    import re

    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    # the 1 GiB copies are the largest dispatches of the runtime's copy kernel
    copy = [k for k in fetch if re.search(r"copy", k, re.I) and "hbm::" not in k]
    if not copy:
        raise SystemExit("no copy kernel in the counter run")
    ck = max(copy, key=lambda k: max(fetch[k]))
    f_scale, w_scale = COPY_BYTES / max(fetch[ck]), COPY_BYTES / max(write.get(ck, [COPY_BYTES]))
    kernels = {}
    mean = lambda v: sum(v) / len(v)
    for prof, sym in PROFILE_KERNELS.items():
        pat = re.compile(r"hbm::" + sym)
        fs = [x for k, v in fetch.items() if pat.search(k) for x in v]
        ws = [x for k, v in write.items() if pat.search(k) for x in v]
        if fs:
            kernels[prof] = mean(fs) * f_scale + (mean(ws) * w_scale if ws else 0.0)
    cmds = ["cd /tmp && rocprofv3 --pmc FETCH_SIZE -f csv -d $GRAFT_REPO_ROOT/gpurun_out/pmc_fetch -o f -- "
            "python $GRAFT_REPO_ROOT/bench.py --traffic-probe",
            "cd /tmp && rocprofv3 --pmc WRITE_SIZE -f csv -d $GRAFT_REPO_ROOT/gpurun_out/pmc_write -o w -- "
            "python $GRAFT_REPO_ROOT/bench.py --traffic-probe",
            "python bench.py --traffic-summarize gpurun_out/pmc_fetch/f_counter_collection.csv "
            "gpurun_out/pmc_write/w_counter_collection.csv"]
    out = {"commands": cmds, "workload": "bench.py default workload, one IMM step", "workload_key": workload,
           "csrc_digest": csrc_digest(), "copy_kernel": ck[:80], "fetch_scale": f_scale, "write_scale": w_scale,
           "unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)", "kernels": kernels}
    json.dump(out, open(out_path, "w"), indent=1)
    print(json.dumps(out))


def traffic_for(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on the current kernels and
    on this workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("csrc_digest") != csrc_digest() or t.get("workload_key") != workload:
        return None
    return t.get("kernels", {}).get(kernel)


def cpu_baseline(g, c, budget_s=12.0):
    """The oracle, as it is, on a bounded prefix of the same RR-set stream (one core)."""
    import oracle

    oracle.build()
    t0 = time.perf_counter()
    og = oracle.Graph(g.n, g.row_ptr, g.dst, g.w if c["prob"] == "EDGE" else None, model=c["model"],
                      prob=c["prob"])
    t_graph = time.perf_counter() - t0
    st = oracle.Store()
    theta, chunk = 0, 1000
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s:
        theta += chunk
        st.extend(og, c["seed"], theta)
    t_sample = time.perf_counter() - t1
    t2 = time.perf_counter()
    oracle.greedy(st, g.n, c["k"])
    t_select = time.perf_counter() - t2
    return {"value": theta / (t_sample + t_select), "unit": "RR sets/s", "cores": 1, "kind": "oracle",
            "sample": f"RR sets 0..{theta - 1} of the same seed-{c['seed']} stream sampled, then greedy "
                      f"k={c['k']} on them; graph transpose ({t_graph:.1f}s) excluded",
            "seconds": t_sample + t_select}


def _instance_graph(inst):
    from synth import graphs as G

    return G.instance_graph(inst)


def batched_graphs(count=256, workers=8):
    """The batched workload's instances and graphs, generated in a process pool.  Call it
    before anything touches the GPU: the pool forks."""
    import concurrent.futures as cf

    from synth import graphs as G

    insts = G.batched_instances(count=count)
    t0 = time.time()
    with cf.ProcessPoolExecutor(workers) as ex:
        graphs = list(ex.map(_instance_graph, insts, chunksize=4))
    log(f"[bench] {count} instance graphs generated ({time.time() - t0:.1f}s), "
        f"{sum(g.m for g in graphs) / 1e6:.1f}M edges in all")
    return insts, graphs


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
    return dict(instances=len(ctxs), tuning=tuning, batched_s=min(tb), plain_s=min(tp), speedup=min(tp) / min(tb),
                identical_results=bool(same), rr_sets=sets, bytes_per_rr=store / max(sets, 1),
                raw_bytes_per_rr=raw / max(sets, 1)), out


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
        "kernels": sorted(({"name": r["name"], "launches": r["launches"], "ms": round(r["total_ms"], 3)}
                           for r in kstats), key=lambda r: -r["ms"])[:8],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_batched(insts, graphs)
    print(json.dumps(res), flush=True)
    for c in ctxs:
        c.close()


def cpu_baseline_batched(insts, graphs, budget_s=12.0):
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
    return {"value": sets / secs, "unit": "RR sets/s", "cores": 1, "kind": "oracle",
            "sample": f"full oracle IMM of the first {done} of {len(insts)} instances ({sets} RR sets, graph "
                      f"transposes included)", "seconds": secs}


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


def main_c5(args, P, torch):
    """The serving loop on the Chung-Lu graph: Poisson arrivals at fractions of the measured
    single-query service rate; p50/p99 latency, throughput, and served == alone."""
    from synth import graphs as G

    wl = WORKLOADS["c5"]
    c = G.C5
    t0 = time.time()
    rp, dst = G.chung_lu_csr(c["n"], c["avg_deg"], c["gamma"], c["gseed"], c["max_deg"], device="cuda")
    torch.cuda.synchronize()
    m = int(dst.numel())
    log(f"[bench] Chung-Lu n={c['n']} m={m} generated on the GPU ({time.time() - t0:.1f}s)")
    ctx = P.Context(0)
    ctx.hbm_load_graph(c["n"], rp, dst, None, "IC", "WC")
    del rp, dst
    torch.cuda.empty_cache()
    ctx.hbm_set_encoding(c["enc"], c["warmup"], c["hot"])
    ctx.hbm_set_hot_density(c["hot_density"])
    ctx.hbm_set_tuning("BLOCK_SETS", 1 << 16)  # short steps: arrivals join within a block's time
    nq = args.queries
    base = G.serving_queries(nq, seed=c["gseed"], rate=1.0)
    # alone: every query of the stream on its own (service times, reference answers)
    alone = {}
    t_alone = []
    for q in base:
        t1 = time.perf_counter()
        s_, g_, st = ctx.hbm_imm(q["k"], q["eps"], q["l"], q["seed"])
        t_alone.append(time.perf_counter() - t1)
        alone[q["q"]] = (s_, g_, st)
    svc = float(np.mean(t_alone))
    log(f"[bench] {nq} queries alone: mean service {svc:.3f}s, max {max(t_alone):.3f}s")
    levels = {}
    identical = True
    for load in args.loads:
        qs = G.serving_queries(nq, seed=c["gseed"], rate=load / svc)
        res, st = serve_level(P, ctx, qs, c["budget"], 16)
        lat = [r["t_done_ms"] - r["t_submit_ms"] for r in res]
        span = (max(r["t_done_ms"] for r in res) - min(r["t_submit_ms"] for r in res)) / 1e3
        ok = all(r["status"] == "OK" for r in res)
        same = ok and all(np.array_equal(r["seeds"], alone[q["q"]][0]) and np.array_equal(r["gains"], alone[q["q"]][1])
                          for r, q in zip(res, qs))
        identical &= same
        sets = sum(r["stats"]["nsets_final"] for r in res if r["status"] == "OK")
        levels[str(load)] = dict(rate_qps=load / svc, p50_ms=pct(lat, 50), p99_ms=pct(lat, 99),
                                 mean_ms=float(np.mean(lat)), makespan_s=span, queries_per_s=nq / span,
                                 rr_sets_per_s=sets / span, served_equals_alone=bool(same),
                                 peak_active=st["peak_active"], preemptions=st["preemptions"],
                                 peak_store_bytes=st["peak_store_bytes"], steps=st["steps"])
        log(f"[bench] load {load}: p50 {levels[str(load)]['p50_ms']:.0f} ms p99 {levels[str(load)]['p99_ms']:.0f} ms "
            f"{nq / span:.2f} q/s peak_active {st['peak_active']} same={same}")
    top = levels[str(max(args.loads))]
    sets_alone = sum(a[2]["nsets_final"] for a in alone.values())
    stores = [a[2]["store"] for a in alone.values()]
    res_line = {
        "metric": METRIC, "value": top["rr_sets_per_s"], "unit": "RR sets/s", "n_gpus": 1, "steps": nq,
        "warmup": 0, "ms_per_step": top["makespan_s"] * 1e3 / nq, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded Chung-Lu digraph; no public dataset)",
        "config": {"workload": wl["name"], "n": c["n"], "m": m, "gamma": c["gamma"], "model": "IC", "prob": "WC",
                   "k": "U{10..200}", "eps": [0.5, 0.2], "queries": nq, "arrivals": "Poisson",
                   "loads": list(args.loads), "store_budget_bytes": c["budget"], "encoding": c["enc"],
                   "hot_min_density": c["hot_density"]},
        "alone": {"mean_service_s": svc, "max_service_s": max(t_alone), "rr_sets_per_s": sets_alone / sum(t_alone)},
        "levels": levels, "served_equals_alone": bool(identical),
        "bytes_per_rr": sum(s_["store_bytes"] for s_ in stores) / max(sets_alone, 1),
        "raw_bytes_per_rr": sum(4 * s_["members"] + 8 * (s_["nsets"] + 1) for s_ in stores) / max(sets_alone, 1),
    }
    print(json.dumps(res_line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain summary of the c2 line")
    ap.add_argument("--queries", type=int, default=24, help="c5: queries per load level")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the workload of the counter runs (one IMM, then a 1 GiB copy) and exit")
    ap.add_argument("--traffic-summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter files into profiles/traffic.json and exit")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 1.0],
                    help="c5: arrival rates as fractions of the measured single-query service rate")
    args = ap.parse_args()
    if args.traffic_summarize:
        return traffic_summarize(*args.traffic_summarize, os.path.join(ROOT, "profiles", "traffic.json"), args.workload)
    if args.traffic_probe:
        return traffic_probe(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU sharding is described in "
                                   "DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2208_00613_amd as P
    from synth import graphs as G

    batched = None
    if args.workload == "c4" or (args.workload == "c2" and not args.no_batched):
        batched = batched_graphs()
    if args.workload == "c4":
        return main_c4(args, P, torch, *batched)
    if args.workload == "c5":
        return main_c5(args, P, torch)
    wl = WORKLOADS[args.workload]
    c = G.CONFIGS[wl["cfg"]]
    t0 = time.time()
    g = G.config_graph(wl["cfg"])
    log(f"[bench] graph {g.name}: n={g.n} m={g.m} ({time.time() - t0:.1f}s)")
    ctx = P.Context(0)
    ctx.load_synth(g, model=c["model"], prob=c["prob"])
    ctx.hbm_set_encoding(c["enc"], c.get("warmup", 0.1), c.get("hot", 0.01))
    torch.cuda.synchronize()
    log("[bench] graph resident in HBM")

    k, eps, l, seed = c["k"], c["eps"], c["l"], c["seed"]
    for i in range(args.warmup):
        seeds, gains, st = ctx.hbm_imm(k, eps, l, seed)
        log(f"[bench] warmup {i}: {st['t_total_ms']:.1f} ms, theta={st['nsets_final']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        seeds, gains, st = ctx.hbm_imm(k, eps, l, seed)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    st = stats[-1]
    nsets = st["nsets_final"]
    store = st["store"]
    out = {
        "metric": METRIC,
        "value": nsets / (ms / 1e3),
        "unit": "RR sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded R-MAT; no public dataset)",
        "config": {"workload": wl["name"], "n": g.n, "m": g.m, "model": c["model"], "prob": c["prob"],
                   "k": k, "eps": eps, "l": l, "encoding": c["enc"], "seed": seed},
        "imm_s": ms / 1e3,
        "theta_final": st["theta_final"],
        "nsets": nsets,
        "rounds": st["rounds"],
        "coverage": st["coverage"],
        "influence": st["influence"],
        "bytes_per_rr": store["store_bytes"] / max(nsets, 1),
        "raw_bytes_per_rr": (4 * store["members"] + 8 * (nsets + 1)) / max(nsets, 1),
        "phase_ms": {"sample_encode": st["t_sample_ms"], "select": st["t_select_ms"]},
    }
    # one profiled step: per-kernel event times on the library's stream, algorithmic work
    ctx.hbm_profile(True)
    ctx.hbm_imm(k, eps, l, seed)
    kstats = ctx.hbm_profile_read()
    ctx.hbm_profile(False)
    out["roofline"] = roofline(kstats, c["model"], c["prob"], args.workload)
    out["kernels"] = sorted(({"name": r["name"], "launches": r["launches"], "ms": round(r["total_ms"], 3)}
                             for r in kstats), key=lambda r: -r["ms"])[:8]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, c)
    ctx.close()
    if args.workload == "c2" and not args.no_batched:
        # the batched form on its own workload, same GPU (256 instances, batched vs plain)
        ctxs = batched_setup(P, *batched)
        out["batched_vs_plain"], _ = batched_vs_plain(P, torch, ctxs, batched[0], reps=1)
        out["batched_vs_plain"]["workload"] = WORKLOADS["c4"]["name"]
        for c4 in ctxs:
            c4.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
