#!/usr/bin/env python3
"""Benchmark of the SCLaP multilevel partitioner on one MI355X.

One step = one full multilevel partition (clustering + contraction per level,
initial partition of the coarsest graph, projection + refinement per level)
of a seeded synthetic graph that is already resident in HBM.  Prints one JSON
line with whole-job edge-visits/s, the roofline of the dominant kernel
(HIP events on the library's stream, algorithmic bytes per launch) and the
CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat24|rmat20|ba14]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    # R-MAT scale 24, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), unit weights, k = 64
    "rmat24": dict(gen="rmat", scale=24, edge_factor=16, k=64, eps=0.03, seed=1, opts={}),
    # R-MAT scale 20, edge factor 16, k = 16
    "rmat20": dict(gen="rmat", scale=20, edge_factor=16, k=16, eps=0.03, seed=1, opts={}),
    # Barabasi-Albert n = 2^14, m = 8, k = 2, one level then refine
    "ba14": dict(gen="ba", n=1 << 14, m=8, k=2, eps=0.03, seed=1, opts={"max_levels": 1}),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_graph(w):
    import numpy as np
    import synth
    if w["gen"] == "rmat":
        g = synth.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
        name = "rmat%d_ef%d_k%d" % (w["scale"], w["edge_factor"], w["k"])
    else:
        g = synth.ba(w["n"], w["m"], seed=w["seed"])
        name = "ba_n%d_m%d_k%d" % (w["n"], w["m"], w["k"])
    # explicit unit weights: int32 CSR with int32 node and edge weights
    g["adjwgt"] = np.ones(len(g["adjncy"]), dtype=np.int32)
    g["vwgt"] = np.ones(g["n"], dtype=np.int32)
    return g, name


def cpu_baseline(g, w):
    """The oracle, as it stands, on a bounded sample: the first sub-round
    (colour 0 of 4) of the first clustering round on the full level-0 graph,
    single thread; then the whole first clustering round (4 sub-rounds) with
    the oracle's node evaluation on all host cores (OpenMP; admission and
    apply sequential, so the labels equal the single-threaded oracle's)."""
    import numpy as np
    import oracle
    n = g["n"]
    U = oracle.cluster_bound(g, w["k"], 18)
    label = np.arange(n, dtype=np.int32)
    wt = g["vwgt"].astype(np.int64)
    t = time.perf_counter()
    moves, visits, ncand = oracle.subround(g, oracle.CLUSTER, 0, 0, 0, 4, w["seed"], U, label, wt)
    dt = time.perf_counter() - t
    one = {"value": visits / dt, "unit": "edge-visits/s", "cores": 1, "kind": "oracle",
           "sample": "oracle sub-round 0 of 4 of clustering round 0 on the full level-0 graph "
                     "(%d edge visits, %.1f s, single thread)" % (visits, dt)}
    threads = oracle.max_threads()
    plabel = np.arange(n, dtype=np.int32)
    pwt = g["vwgt"].astype(np.int64)
    t = time.perf_counter()
    pvisits = 0
    for sub in range(4):
        _, v = oracle.subround_par(g, oracle.CLUSTER, 0, 0, sub, 4, w["seed"], U, plabel, pwt, threads=threads)
        pvisits += v
        if sub == 0:
            assert np.array_equal(plabel, label), "parallel oracle sub-round differs"
    pdt = time.perf_counter() - t
    allc = {"value": pvisits / pdt, "unit": "edge-visits/s", "cores": threads, "kind": "oracle",
            "sample": "oracle clustering round 0 (4 sub-rounds) on the full level-0 graph with the node evaluation "
                      "on %d OpenMP threads (%d edge visits, %.1f s)" % (threads, pvisits, pdt)}
    return one, allc


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter record in
    profiles/, or None if there is none or the kernel source changed since."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md")):
        for line in open(path):
            if not line.startswith("machine-readable:"):
                continue
            kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
            if kv.get("kernel") != kernel or kv.get("workload", workload) != workload:
                continue
            src = os.path.join(ROOT, kv["source"])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("sha256"):
                return None
            return float(kv["traffic_bytes_per_launch"])
    return None


def batch_comparison(ngraphs, seed, log_lo, log_hi, extra=None):
    """Batched vs plain on the same device-resident mix: all graphs in one
    batched call, then each graph by itself through the one-graph entry
    point; per-graph parts and cuts must be identical."""
    import numpy as np
    import torch
    import synth
    import paper_1404_4797_amd as sc
    t = time.time()
    gs = synth.batch_mix(ngraphs, seed=seed, n_lo_log2=log_lo, n_hi_log2=log_hi)
    ks = [g["k"] for g in gs]
    eps = [g["eps"] for g in gs]
    seeds = [g["seed"] for g in gs]
    u, nb = sc.union(gs)
    log("batch mix: %d graphs, n=%d S=%d generated in %.1fs" % (ngraphs, u["n"], int(u["xadj"][-1]),
                                                               time.time() - t))
    du = sc.to_device(u, "cuda")
    dgs = [sc.to_device(g, "cuda") for g in gs]
    part = torch.empty(max(u["n"], 1), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    extra = extra or {}
    r = sc.partition_batch_dev(du, nb, ks, eps, seeds, part=part, stream=stream, **extra)  # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sc.partition_batch_dev(du, nb, ks, eps, seeds, part=part, stream=stream, **extra)
    torch.cuda.synchronize()
    t_default = time.perf_counter() - t0
    ref_part = part.clone()
    # tuning options (degree thresholds, so LDS table sizes per degree range,
    # and graph capture) searched on the union by the library's autotuner
    t0 = time.perf_counter()
    o = sc.autotune_dev(du, int(np.median(ks)), stream=stream, **extra)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    tuned = {"lane_max_degree": o.lane_max_degree, "wave_max_degree": o.wave_max_degree,
             "block_max_degree": o.block_max_degree, "graph_capture": o.graph_capture,
             "block_table": o.block_table}
    r = sc.partition_batch_dev(du, nb, ks, eps, seeds, part=part, stream=stream, opts=o)  # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sc.partition_batch_dev(du, nb, ks, eps, seeds, part=part, stream=stream, opts=o)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = bool(torch.equal(part, ref_part))
    log("batched: %.1f ms default thresholds, %.1f ms tuned %s (tuning %.1f ms), identical=%s"
        % (t_default * 1e3, t_batch * 1e3, tuned, t_tune * 1e3, same))
    bpart = part.cpu().numpy()
    t_plain = 0.0
    visits_plain = 0
    for i, dg in enumerate(dgs):
        p = torch.empty(max(gs[i]["n"], 1), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q = sc.partition_dev(dg, ks[i], eps[i], seeds[i], part=p, stream=stream, **extra)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        visits_plain += q["stats"]["visits"]
        if q["cut"] != int(r["cut"][i]) or not np.array_equal(p.cpu().numpy()[:gs[i]["n"]],
                                                              bpart[nb[i]:nb[i + 1]]):
            same = False
    log("plain: %.1f ms for %d graphs, identical=%s" % (t_plain * 1e3, ngraphs, same))
    return {"graphs": ngraphs, "n_log2_range": [log_lo, log_hi], "n": u["n"], "S": int(u["xadj"][-1]),
            "batched_ms": round(t_batch * 1e3, 3), "batched_default_options_ms": round(t_default * 1e3, 3),
            "tuned_options": tuned, "tuned_vs_default": round(t_default / t_batch, 4),
            "tuning_ms": round(t_tune * 1e3, 3), "plain_ms": round(t_plain * 1e3, 3),
            "batched_graphs_per_s": ngraphs / t_batch, "plain_graphs_per_s": ngraphs / t_plain,
            "speedup": t_plain / t_batch, "identical_parts_and_cuts": same,
            "batched_edge_visits": r["stats"]["visits"], "plain_edge_visits": visits_plain,
            "levels_max": r["stats"]["levels"],
            "batched_phase_ms": {"coarsen": round(r["stats"]["ms_coarsen"], 3),
                                 "initial": round(r["stats"]["ms_initial"], 3),
                                 "refine": round(r["stats"]["ms_refine"], 3)}}


def mesh_runs(log2n, k, eps, seed):
    """The paper's mesh-type families (delX, rggX with radius 0.55 sqrt(ln n/n))
    at n = 2^log2n: one warm-up and one timed partition each."""
    import numpy as np
    import torch
    import synth
    import paper_1404_4797_amd as sc
    out = {}
    for name, make in (("del%d" % log2n, lambda: synth.delaunay(1 << log2n, seed=seed)),
                       ("rgg%d_paper" % log2n, lambda: synth.rgg_paper(1 << log2n, seed=seed))):
        t = time.time()
        g = make()
        log("mesh %s: n=%d S=%d generated in %.1fs" % (name, g["n"], int(g["xadj"][-1]), time.time() - t))
        d = sc.to_device(g, "cuda")
        part = torch.empty(g["n"], dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream()
        sc.partition_dev(d, k, eps, seed, part=part, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sc.partition_dev(d, k, eps, seed, part=part, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        st = r["stats"]
        out[name] = {"n": g["n"], "S": int(g["xadj"][-1]), "k": k, "ms": round(ms, 3), "cut": r["cut"],
                     "status": r["status"], "levels": st["levels"], "level_n": st["level_n"],
                     "edge_visits": st["visits"], "edge_visits_per_s": st["visits"] / (ms / 1e3),
                     "max_block_weight": int(np.max(r["block_weights"]))}
        log("mesh %s: %.1f ms, cut %d, levels %d" % (name, ms, r["cut"], st["levels"]))
        del d, part
    return out


def serve_benchmark(nreq, log_lo, log_hi, fracs, slots=3, max_batch=64):
    """Poisson arrivals of partition requests (the batch mix's graph
    distribution, n log-uniform in [2^log_lo, 2^log_hi], seed 7) at fixed
    rates, given as multiples of the plain path's throughput on the same
    requests; reports p50/p99 latency (arrival to result) with the queueing
    and service parts of the slowest requests, graphs/s of the
    continuous-batching server, and the batched path (max_batch graphs per
    call) on the same requests.  Every served and batched result must equal
    the plain path's part of that request, node for node."""
    import threading
    import numpy as np
    import torch
    import synth
    import paper_1404_4797_amd as sc
    t = time.time()
    gs = synth.batch_mix(nreq, seed=7, n_lo_log2=log_lo, n_hi_log2=log_hi,
                         progress=lambda i: log("serve mix: %d graphs generated" % i))
    ntot = sum(g["n"] for g in gs)
    log("serve mix: %d requests, n=%d generated in %.1fs" % (nreq, ntot, time.time() - t))
    # plain path: one graph per call, the graph already on the device
    plain_part, plain_cut = [], []
    t_plain = 0.0
    stream = torch.cuda.current_stream()
    for i, g in enumerate(gs):
        d = sc.to_device(g, "cuda")
        p = torch.empty(max(g["n"], 1), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sc.partition_dev(d, g["k"], g["eps"], g["seed"], part=p, stream=stream)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        plain_part.append(p[:g["n"]].cpu().numpy())
        plain_cut.append(r["cut"])
        del d, p
        if (i + 1) % 200 == 0:
            log("plain: %d of %d requests" % (i + 1, nreq))
    plain_gps = nreq / t_plain
    log("plain: %.1f graphs/s on %d requests" % (plain_gps, nreq))
    # batched path: consecutive groups of max_batch requests, one call each
    t_batch = 0.0
    batch_same = True
    for b0 in range(0, nreq, max_batch):
        grp = gs[b0:b0 + max_batch]
        u, nb = sc.union(grp)
        du = sc.to_device(u, "cuda")
        part = torch.empty(max(u["n"], 1), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sc.partition_batch_dev(du, nb, [g["k"] for g in grp], [g["eps"] for g in grp],
                                   [g["seed"] for g in grp], part=part, stream=stream)
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
        bp = part.cpu().numpy()
        for j in range(len(grp)):
            batch_same &= bool(np.array_equal(bp[nb[j]:nb[j + 1]], plain_part[b0 + j])) and \
                int(r["cut"][j]) == plain_cut[b0 + j]
        del du, part
    log("batched: %.1f graphs/s in groups of %d, identical=%s" % (nreq / t_batch, max_batch, batch_same))
    rng = np.random.default_rng(7)
    runs = []
    serve_same = True
    with sc.Server(slots=slots, max_batch=max_batch) as sv:
        sv.wait(sv.submit(gs[0], gs[0]["k"], gs[0]["eps"], gs[0]["seed"]))  # warm up the workers
        for f in fracs:
            qps = f * plain_gps
            gaps = rng.exponential(1.0 / qps, size=nreq)
            ids = [None] * nreq

            def producer():
                t_next = time.perf_counter()
                for i, g in enumerate(gs):
                    t_next += gaps[i]
                    dt = t_next - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                    ids[i] = sv.submit(g, g["k"], g["eps"], g["seed"])

            th = threading.Thread(target=producer)
            th.start()
            th.join()
            res = [sv.wait(i) for i in ids]
            same = all(r["cut"] == plain_cut[i] and np.array_equal(r["part"], plain_part[i])
                       for i, r in enumerate(res))
            serve_same &= same
            lat = np.array([r["done_ms"] - r["submit_ms"] for r in res])
            wait = np.array([r["start_ms"] - r["submit_ms"] for r in res])
            service = np.array([r["done_ms"] - r["start_ms"] for r in res])
            span = (max(r["done_ms"] for r in res) - min(r["submit_ms"] for r in res)) / 1000.0
            slow = np.argsort(lat)[-max(1, nreq // 100):]  # the requests at or above p99
            runs.append({"rate_vs_plain": f, "offered_qps": round(qps, 2), "graphs_per_s": round(nreq / span, 2),
                         "p50_ms": round(float(np.percentile(lat, 50)), 2),
                         "p99_ms": round(float(np.percentile(lat, 99)), 2),
                         "mean_batch": round(float(np.mean([r["batch_size"] for r in res])), 2),
                         "identical_parts": bool(same),
                         "tail": {"requests": int(len(slow)),
                                  "median_n": int(np.median([gs[i]["n"] for i in slow])),
                                  "median_n_all": int(np.median([g["n"] for g in gs])),
                                  "mean_wait_ms": round(float(wait[slow].mean()), 2),
                                  "mean_service_ms": round(float(service[slow].mean()), 2),
                                  "mean_batch": round(float(np.mean([res[i]["batch_size"] for i in slow])), 2)}})
            log("serve at %.1fx plain (%.1f qps): %s" % (f, qps, runs[-1]))
    return {"requests": nreq, "n_log2_range": [log_lo, log_hi], "nodes": int(ntot),
            "plain_graphs_per_s": round(plain_gps, 2), "batched_graphs_per_s": round(nreq / t_batch, 2),
            "batch_size": max_batch, "identical_parts_batched": bool(batch_same),
            "identical_parts_served": bool(serve_same), "runs": runs}


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: %d bytes read, %d bytes written" % (a.numel() * 4, b.numel() * 4))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=INT",
                    help="extra sclap_options field for the timed partitions (e.g. skip_quiet=1)")
    ap.add_argument("--mesh-log2", type=int, default=20,
                    help="log2 n of the Delaunay and RGG (paper radius) runs (0: skip)")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the V-cycle / degree-order runs after the timed steps")
    ap.add_argument("--copy-calib", type=int, default=0, help="bytes for a plain copy kernel (counter scaling)")
    ap.add_argument("--no-kernel-timing", dest="kernel_timing", action="store_false",
                    help="no HIP events around the dominant kernel in the timed steps (no roofline)")
    ap.add_argument("--batch-graphs", type=int, default=512, help="graphs in the batched-vs-plain comparison (0: skip)")
    ap.add_argument("--batch-log2", type=int, nargs=2, default=[10, 18], help="log2 range of n in the batch")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests per serving run (0: skip); the Poisson serving workload has 2000")
    ap.add_argument("--serve-log2", type=int, nargs=2, default=[10, 20], help="log2 range of n of the requests")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[0.5, 0.8],
                    help="arrival rates as multiples of the plain path's graphs/s")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the partitioner runs on one GPU; --gpus %d is not supported "
              "(sharding over several GPUs is not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1404_4797_amd as sc

    w = WORKLOADS[args.workload]
    t = time.time()
    g, name = make_graph(w)
    n, S = g["n"], int(g["xadj"][-1])
    log("workload %s: n=%d S=%d generated in %.1fs" % (name, n, S, time.time() - t))
    torch.cuda.set_device(0)
    d = sc.to_device(g, "cuda")
    part = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    extra = {}
    for kv in args.opt:
        key, val = kv.split("=", 1)
        extra[key] = int(val)
    opts = sc.default_options(**w["opts"], **extra)
    torch.cuda.synchronize()
    if args.copy_calib:
        copy_calibration(args.copy_calib)

    for i in range(args.warmup):
        r = sc.partition_dev(d, w["k"], w["eps"], w["seed"], part=part, stream=stream, opts=opts)
        log("warmup %d: cut=%d levels=%d" % (i, r["cut"], r["stats"]["levels"]))
    torch.cuda.synchronize()
    # one step with events around every launch, outside the timed region: the
    # per-kernel breakdown and the dominant kernel (events cost device time
    # between launches, so the timed steps carry them for that kernel alone)
    sc.profile_begin()
    r_prof = sc.partition_dev(d, w["k"], w["eps"], w["seed"], part=part, stream=stream, opts=opts)
    torch.cuda.synchronize()
    kstats = sc.profile_end()
    modeled = {k: v for k, v in kstats.items() if v["bytes"] > 0 and v["launches"] > 0}
    dom = max(modeled, key=lambda k: modeled[k]["ms"]) if modeled else None
    log("profiled step: cut=%d, dominant kernel %s" % (r_prof["cut"], dom))

    if args.kernel_timing:
        sc.profile_begin(only=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        r = sc.partition_dev(d, w["k"], w["eps"], w["seed"], part=part, stream=stream, opts=opts)
        results.append(r)
        log("step %d: cut=%d" % (i, r["cut"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kdom = sc.profile_end() if args.kernel_timing else {}
    ms_per_step = (t1 - t0) * 1000.0 / max(args.steps, 1)
    r = results[-1]
    st = r["stats"]
    assert all(x["cut"] == r["cut"] for x in results + [r_prof]), "steps disagree"
    visits = st["visits"]
    value = visits / (ms_per_step / 1000.0)

    # dominant kernel with an algorithmic byte model, timed live over the
    # timed steps
    roofline = None
    if dom and dom in kdom and kdom[dom]["launches"] > 0:
        ks = kdom[dom]
        avg_ms = ks["ms"] / ks["launches"]
        gbs = ks["bytes"] / (ks["ms"] / 1000.0) / 1e9
        traffic = recorded_traffic(dom, name)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_GBps": round(traffic / avg_ms / 1e6, 1) if traffic else None,
                    "avg_launch_ms": round(avg_ms, 5), "bytes_per_launch": ks["bytes"] / ks["launches"],
                    "launches": ks["launches"] // max(args.steps, 1)}
    # per-kernel breakdown of the one fully profiled step
    total_k_ms = sum(v["ms"] for v in kstats.values())
    kernels = {k: {"ms_per_step": round(v["ms"], 3),
                   "share": round(v["ms"] / total_k_ms, 4) if total_k_ms else 0,
                   "launches_per_step": v["launches"],
                   "GBps": round(v["bytes"] / (v["ms"] / 1000.0) / 1e9, 1) if v["bytes"] and v["ms"] else None}
               for k, v in sorted(kstats.items(), key=lambda kv: -kv[1]["ms"])}
    lp_gb = sum(v["bytes"] for k, v in kstats.items()
                if k.startswith("lp_eval") or k.startswith("lp_refine")) / 1e9
    # the whole label-propagation phase against the HBM roofline: per round
    # executed at level l, 24 B per node and 12 B per slot scanned (a round's
    # minimal traffic), over the wall time of all rounds
    lp_nodes = sum(st["level_n"][l] * st["cluster_rounds"][l] for l in range(len(st["cluster_rounds"])))
    lp_nodes += sum(st["level_n"][l] * st["refine_rounds"][l] for l in range(len(st["refine_rounds"])))
    lp_bytes = 24.0 * lp_nodes + 12.0 * visits
    lp_phase = {"bytes_per_step": lp_bytes, "ms": round(st["ms_lp"], 3),
                "achieved_GBps": round(lp_bytes / (st["ms_lp"] / 1e3) / 1e9, 1),
                "frac": round(lp_bytes / (st["ms_lp"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "edge_visits_per_s": visits / (st["ms_lp"] / 1e3)}

    # the access that bounds evaluation: one neighbour-label gather per slot,
    # measured by the library's probe kernel on this graph (4-byte labels as
    # in clustering, 1-byte labels as in refinement); the label-propagation
    # rounds' visits at those rates bound their time from below
    gather = None
    if S > 0:
        g4 = sc.gather_probe_dev(d, 4, reps=3, stream=stream)
        g1 = sc.gather_probe_dev(d, 1, reps=3, stream=stream)
        r4, r1 = S / (g4 / 1e3), S / (g1 / 1e3)
        cvis = sum(st["level_S"][l] * st["cluster_rounds"][l] for l in range(len(st["cluster_rounds"])))
        rvis = visits - cvis
        floor_ms = (cvis / r4 + rvis / r1) * 1e3
        lp_ms = st["ms_lp"]
        gather = {"ms_per_pass_i32": round(g4, 3), "ms_per_pass_u8": round(g1, 3),
                  "G_gathers_per_s_i32": round(r4 / 1e9, 1), "G_gathers_per_s_u8": round(r1 / 1e9, 1),
                  "lp_ms_at_ceiling": round(floor_ms, 1), "lp_ms": round(lp_ms, 1),
                  "frac": round(floor_ms / lp_ms, 3),
                  "lp_bytes_frac_at_ceiling": round(lp_bytes / (floor_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("gather ceiling: %.1f G/s (int32 labels), %.1f G/s (byte labels); LP %.1f ms vs %.1f ms at the ceiling"
            % (r4 / 1e9, r1 / 1e9, lp_ms, floor_ms))

    out = {
        "metric": "SCLaP edge-visits/s & partition time; batched vs plain graphs/s, same cut",
        "value": value, "unit": "edge-visits/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": name, "n": n, "S": S, "k": w["k"], "eps": w["eps"], "seed": w["seed"],
                   "coarsen_rounds": opts.coarsen_rounds, "refine_rounds": opts.refine_rounds,
                   "subrounds": opts.subrounds, "max_levels": opts.max_levels},
        "partition_ms": ms_per_step, "edge_visits_per_step": visits, "cut": r["cut"],
        "max_block_weight": int(np.max(r["block_weights"])), "status": r["status"],
        "levels": st["levels"], "level_n": st["level_n"], "level_S": st["level_S"],
        "cluster_rounds": st["cluster_rounds"],
        "refine_rounds": st["refine_rounds"],
        "phase_ms": {"coarsen": st["ms_coarsen"], "initial": st["ms_initial"], "refine": st["ms_refine"],
                     "lp": st["ms_lp"]},
        "lp_eval_GB_per_step": round(lp_gb, 3),
        "roofline": roofline, "lp_phase_roofline": lp_phase, "gather_ceiling": gather, "kernels": kernels,
        "kernels_from": "one step with events around every launch, outside the timed steps",
    }
    if args.variants:
        # the paper's quality levers on the same workload, one timed run each
        var = {}
        for vname, kw in (("vcycles2", dict(vcycles=2)), ("degree_order", dict(degree_order=1)),
                          ("degree_order_vcycles2", dict(degree_order=1, vcycles=2)),
                          ("device_initial", dict(initial_partitioner=1))):
            vo = sc.default_options(**w["opts"], **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q = sc.partition_dev(d, w["k"], w["eps"], w["seed"], part=part, stream=stream, opts=vo)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1000.0
            var[vname] = {"ms": round(ms, 3), "cut": q["cut"], "cut_vs_default": round(q["cut"] / r["cut"], 5),
                          "status": q["status"], "edge_visits": q["stats"]["visits"],
                          "max_block_weight": int(np.max(q["block_weights"]))}
            log("variant %s: %.1f ms cut=%d (%.4f of the default cut)" % (vname, ms, q["cut"], q["cut"] / r["cut"]))
        out["variants"] = var
    if args.mesh_log2 > 0:
        out["mesh"] = mesh_runs(args.mesh_log2, w["k"], w["eps"], w["seed"])
    if args.batch_graphs > 0:
        out["batched"] = batch_comparison(args.batch_graphs, 0, args.batch_log2[0], args.batch_log2[1], extra)
    if args.serve_requests > 0:
        out["serving"] = serve_benchmark(args.serve_requests, args.serve_log2[0], args.serve_log2[1],
                                         args.serve_rates)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        out["cpu_baseline"], out["cpu_baseline_all_cores"] = cpu_baseline(g, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
