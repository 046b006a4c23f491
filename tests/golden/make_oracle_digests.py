"""Writes oracle_digests.json: digests of the CPU oracle's multilevel output
on the seeded benchmark workloads, for GPU parity tests at sizes where the
oracle takes too long to run inside a test.

Calls only the oracle and the input generators:
    python tests/golden/make_oracle_digests.py          # workloads not yet stored
    python tests/golden/make_oracle_digests.py --all    # every workload
    python tests/golden/make_oracle_digests.py --only rmat24_ef16_k64
    python tests/golden/make_oracle_digests.py --batch  # batch_mix_digests.json

The 2^24 R-MAT takes about an hour on one core and about 30 GB of memory
(the oracle's symmetry check and contraction sort triples of all slots).
The batch mix (512 graphs) runs its graphs on several processes.
"""
import hashlib
import json
import multiprocessing
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

WORKLOADS = {
    # Barabasi-Albert n=2^14, m=8, unit weights; one level then refine; k=2
    "ba14_m8_k2_onelevel": dict(gen=("ba", dict(n=1 << 14, m=8, seed=1)), k=2, eps=0.03, seed=1,
                                opts=dict(max_levels=1)),
    # R-MAT scale 20, edge factor 16, (0.57, 0.19, 0.19, 0.05); full multilevel; k=16
    "rmat20_ef16_k16": dict(gen=("rmat", dict(scale=20, edge_factor=16, seed=1)), k=16, eps=0.03, seed=1,
                            opts=dict()),
    # Delaunay triangulation of 2^18 uniform points (the paper's delX family); k=16
    "del18_k16": dict(gen=("del", dict(n=1 << 18, seed=1)), k=16, eps=0.03, seed=1, opts=dict()),
    # the same with two multilevel cycles (Section 4.4, iterated V-cycles)
    "rmat20_ef16_k16_vcycles2": dict(gen=("rmat", dict(scale=20, edge_factor=16, seed=1)), k=16, eps=0.03,
                                     seed=1, opts=dict(vcycles=2)),
    # R-MAT scale 24, edge factor 16: the web-scale single graph of the benchmark, k=64, default options
    "rmat24_ef16_k64": dict(gen=("rmat", dict(scale=24, edge_factor=16, seed=1)), k=64, eps=0.03, seed=1,
                            opts=dict()),
}

# the benchmark's batched mix: 512 graphs, n log-uniform in [2^10, 2^18], mix seed 0
BATCH = dict(count=512, seed=0, n_lo_log2=10, n_hi_log2=18)


def make_graph(spec):
    kind, kw = spec
    if kind == "del":
        return synth.delaunay(**kw)
    return synth.ba(**kw) if kind == "ba" else synth.rmat(**kw)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


_MIX = None


def _mix_one(i):
    g = _MIX[i]
    r = oracle.partition(g, g["k"], g["eps"], g["seed"])
    return i, {"n": int(g["n"]), "S": int(g["xadj"][-1]), "k": g["k"], "eps": g["eps"], "seed": g["seed"],
               "kind": g["kind"], "input_sha256": digest(g["adjncy"]),
               "part_sha256": digest(r["part"].astype(np.int32)), "cut": r["cut"],
               "block_weights": r["block_weights"].tolist(), "status": r["status"], "levels": r["levels"],
               "level_n": r["level_n"], "visits": r["visits"]}


def batch_main(workers):
    """Per-graph oracle digests of the benchmark's batched mix."""
    global _MIX
    path = os.path.join(HERE, "batch_mix_digests.json")
    t = time.time()
    _MIX = synth.batch_mix(**BATCH)
    print("mix generated in %.1fs" % (time.time() - t), flush=True)
    graphs = [None] * len(_MIX)
    order = sorted(range(len(_MIX)), key=lambda i: -int(_MIX[i]["xadj"][-1]))  # largest first
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        for done, (i, d) in enumerate(pool.imap_unordered(_mix_one, order)):
            graphs[i] = d
            if done % 32 == 0:
                print("%d/%d graphs (%.0fs)" % (done + 1, len(order), time.time() - t), flush=True)
    out = {"note": "Per-graph digests of the oracle's output on the batched mix; regenerate with this script "
                   "(--batch).", "mix": BATCH, "graphs": graphs}
    with open(path, "w") as f:
        json.dump(out, f, indent=0)


def main():
    if "--batch" in sys.argv:
        batch_main(int(os.environ.get("DIGEST_WORKERS", "6")))
        return
    path = os.path.join(HERE, "oracle_digests.json")
    out = {"note": "Digests of the oracle's output; regenerate with this script.", "workloads": {}}
    if "--all" not in sys.argv and os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    only = sys.argv[sys.argv.index("--only") + 1] if "--only" in sys.argv else None
    for name, w in WORKLOADS.items():
        if only is not None and name != only:
            continue
        if name in out["workloads"] and only is None:
            continue
        g = make_graph(w["gen"])
        t = time.time()
        r = oracle.partition(g, w["k"], w["eps"], w["seed"], **w["opts"])
        print("%s: %.1fs cut=%d levels=%d" % (name, time.time() - t, r["cut"], r["levels"]), flush=True)
        out["workloads"][name] = {
            "graph": {"kind": w["gen"][0], **w["gen"][1]}, "k": w["k"], "eps": w["eps"], "seed": w["seed"],
            "opts": w["opts"], "n": int(g["n"]), "S": int(g["xadj"][-1]),
            "input_sha256": digest(g["adjncy"]),
            "part_sha256": digest(r["part"].astype(np.int32)), "cut": r["cut"],
            "block_weights": r["block_weights"].tolist(), "status": r["status"], "levels": r["levels"],
            "level_n": r["level_n"], "level_S": [int(x) for x in r["level_S"]], "visits": r["visits"],
            "cluster_rounds": r["cluster_rounds"], "refine_rounds": r["refine_rounds"],
        }
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
