"""Batched partitioning: many graphs in one CSR, one multilevel pass.

Each graph's result from the batched entry point must equal the CPU oracle's
partition of that graph alone (and so the plain one-graph entry point's),
bit for bit: blocks, cut, block weights and the number of levels kept.  The
mixes cover graphs that stop coarsening at different levels, graphs too small
to coarsen, empty and edgeless graphs, k = 1, weighted edges and nodes, and
per-graph k, eps and seed.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sc():
    import paper_1404_4797_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m.load()
    return m


def say(*a):
    print(*a, flush=True)


def edgeless(n):
    return {"n": n, "xadj": np.zeros(n + 1, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32),
            "adjwgt": np.zeros(0, dtype=np.int32), "vwgt": np.ones(n, dtype=np.int32)}


def node_weighted(g, seed):
    rng = np.random.default_rng(seed)
    h = dict(g)
    h["vwgt"] = rng.integers(0, 5, size=g["n"]).astype(np.int32)
    return h


def mix_small():
    gs = [synth.ba(3000, 4, seed=101, weighted=True),
          synth.rmat(11, 12, seed=102, weighted=True),
          synth.rgg(2500, seed=103, weighted=True),
          edgeless(0),
          synth.ba(40, 2, seed=104),
          edgeless(300),
          node_weighted(synth.rmat(12, 8, seed=105, weighted=True, n=3000), 7),
          synth.rgg(800, seed=106),
          synth.ba(5000, 8, seed=107, weighted=True),
          synth.from_edges(6, [(0, 1), (1, 2), (3, 4)])]
    ks = [4, 16, 2, 3, 1, 8, 5, 2, 64, 2]
    eps = [0.03, 0.01, 0.05, 0.03, 0.03, 0.0, 0.03, 0.05, 0.03, 0.03]
    seeds = [1000 + i for i in range(len(gs))]
    return gs, ks, eps, seeds


def check_against_oracle(r, gs, ks, eps, seeds, **opts):
    for i, g in enumerate(gs):
        ref = oracle.partition(g, ks[i], eps[i], seeds[i], **opts)
        got = r["graphs"][i]
        assert np.array_equal(got["part"], ref["part"]), i
        assert got["cut"] == ref["cut"], i
        assert np.array_equal(got["block_weights"], ref["block_weights"]), i
        assert got["levels"] == len(ref["level_n"]) - 1, i


@pytest.mark.parametrize("opts", [dict(coarsest_nodes=200), dict(coarsest_nodes=50, max_levels=2),
                                  dict(max_levels=1), dict(coarsest_nodes=100000),
                                  dict(coarsest_nodes=200, lane_max_degree=2, wave_max_degree=8,
                                       block_max_degree=24, select_small_max=1),
                                  dict(coarsest_nodes=200, skip_quiet=-1)])
def test_batch_matches_oracle_per_graph(sc, opts):
    gs, ks, eps, seeds = mix_small()
    say("batch", opts)
    r = sc.partition_batch(gs, ks, eps, seeds, **opts)
    check_against_oracle(r, gs, ks, eps, seeds, **{k: v for k, v in opts.items()
                                                   if k in ("coarsest_nodes", "max_levels")})


def test_batch_equals_plain_entry_point(sc):
    gs, ks, eps, seeds = mix_small()
    r = sc.partition_batch(gs, ks, eps, seeds, coarsest_nodes=200)
    for i, g in enumerate(gs):
        if g["n"] == 0:
            continue
        p = sc.partition(g, ks[i], eps[i], seeds[i], coarsest_nodes=200)
        assert np.array_equal(p["part"], r["graphs"][i]["part"]) and p["cut"] == r["graphs"][i]["cut"]


def test_batch_device_entry_point(sc):
    gs, ks, eps, seeds = mix_small()
    u, nb = sc.union(gs)
    d = sc.to_device(u, "cuda")
    r = sc.partition_batch_dev(d, nb, ks, eps, seeds, coarsest_nodes=200)
    h = sc.partition_batch(gs, ks, eps, seeds, coarsest_nodes=200)
    part = r["part"].cpu().numpy()
    for i in range(len(gs)):
        assert np.array_equal(part[nb[i]:nb[i + 1]], h["graphs"][i]["part"])
        assert r["cut"][i] == h["graphs"][i]["cut"]


def test_batch_mix_generator_slice(sc):
    # the batched workload's generator (BA, R-MAT, RGG; weighted; per-graph k,
    # eps, seed), on a small size range so the oracle finishes quickly
    gs = synth.batch_mix(12, seed=3, n_lo_log2=8, n_hi_log2=13)
    ks = [g["k"] for g in gs]
    eps = [g["eps"] for g in gs]
    seeds = [g["seed"] for g in gs]
    r = sc.partition_batch(gs, ks, eps, seeds, coarsest_nodes=500)
    check_against_oracle(r, gs, ks, eps, seeds, coarsest_nodes=500)


def test_batch_rejects_edges_between_graphs(sc):
    # two paths 0-1-2-3-4 and 5-6-7-8-9 plus the edge (4, 5) across them
    edges = [(i, i + 1) for i in range(4)] + [(i, i + 1) for i in range(5, 9)] + [(4, 5)]
    u = synth.from_edges(10, edges)
    with pytest.raises(sc.SclapError) as e:
        sc.partition_batch_union(u, [0, 5, 10], [2, 2], [0.03, 0.03], [1, 2])
    assert e.value.status == -1
    with pytest.raises(sc.SclapError):  # node bases must cover n
        sc.partition_batch_union(u, [0, 5, 9], [2, 2], [0.03, 0.03], [1, 2])


def test_autotuned_thresholds_leave_results_unchanged(sc):
    gs, ks, eps, seeds = mix_small()
    u, nb = sc.union(gs)
    d = sc.to_device(u, "cuda")
    o = sc.autotune_dev(d, int(np.median(ks)), coarsest_nodes=200)
    # the coordinate search's value grids
    assert o.lane_max_degree in (4, 8, 16) and o.wave_max_degree in (32, 64, 128, 256)
    assert o.block_max_degree in (1024, 2048, 4096, 8192) and o.graph_capture in (-1, 0, 1)
    assert o.block_table in (10240, 16384)
    assert o.coarsest_nodes == 200
    tuned = sc.partition_batch_dev(d, nb, ks, eps, seeds, opts=o)
    plain = sc.partition_batch_dev(d, nb, ks, eps, seeds, coarsest_nodes=200)
    assert torch.equal(tuned["part"], plain["part"])
    assert np.array_equal(tuned["cut"], plain["cut"]) and np.array_equal(tuned["block_weights"], plain["block_weights"])


def test_batch_mix512_oracle_digests(sc, golden_dir):
    # The benchmark's batched workload (512 graphs, n log-uniform in
    # [2^10, 2^18], a third each of BA, R-MAT and RGG, per-graph k, eps and
    # seed) in exactly the benchmark's call: every graph's blocks, cut and
    # block weights equal the stored digests of the oracle run on that graph
    # alone (tests/golden/make_oracle_digests.py --batch).
    import hashlib
    import json
    import os
    with open(os.path.join(golden_dir, "batch_mix_digests.json")) as f:
        gold = json.load(f)
    say("generating the 512-graph batch mix")
    gs = synth.batch_mix(**gold["mix"])
    assert len(gs) == len(gold["graphs"])
    for g, d in zip(gs, gold["graphs"]):
        assert int(g["n"]) == d["n"] and hashlib.sha256(g["adjncy"].tobytes()).hexdigest() == d["input_sha256"]
    u, nb = sc.union(gs)
    du = sc.to_device(u, "cuda")
    part = torch.empty(max(u["n"], 1), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    ks = [g["k"] for g in gs]
    say("batched partition of %d graphs, n=%d" % (len(gs), u["n"]))
    r = sc.partition_batch_dev(du, nb, ks, [g["eps"] for g in gs], [g["seed"] for g in gs], part=part,
                               stream=stream)
    torch.cuda.synchronize()
    p = part.cpu().numpy()
    kb = np.concatenate([[0], np.cumsum(ks)])
    bad = []
    for i, d in enumerate(gold["graphs"]):
        pi = np.ascontiguousarray(p[nb[i]:nb[i + 1]])
        ok = (hashlib.sha256(pi.tobytes()).hexdigest() == d["part_sha256"] and int(r["cut"][i]) == d["cut"]
              and r["block_weights"][kb[i]:kb[i + 1]].tolist() == d["block_weights"]
              and int(r["levels"][i]) == d["levels"])
        if not ok:
            bad.append(i)
    assert not bad, "graphs differing from the oracle: %s" % bad[:20]
