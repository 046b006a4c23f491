"""Full-size checks on the benchmark graph (R-MAT scale 24, edge factor 16,
k = 64), in the launch configuration the benchmark times.

The oracle cannot run the whole path at this size, so it checks sampled
outputs one by one: with one sub-round (every node in colour 0) each node's
decision is a function of the initial state, which the oracle evaluates per
node; with unit weights a target that rejected a candidate must have admitted
exactly bound - w(t) nodes.  The full partition is checked through
properties that hold at any size: block weights and cut recomputed from the
output, balance, determinism.
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


@pytest.fixture(scope="module")
def big(sc):
    print("generating R-MAT scale 24", flush=True)
    g = synth.rmat(24, 16, seed=1)
    return g, sc.to_device(g, "cuda")


def sample_nodes(g, count, seed):
    deg = np.diff(g["xadj"])
    rng = np.random.default_rng(seed)
    pos = np.flatnonzero(deg > 0)
    hubs = np.argsort(deg)[-64:]  # the heaviest rows take the hub path
    return np.unique(np.concatenate([rng.choice(pos, count, replace=False), hubs]))


def check_subround(g, phase, bound, before, after, w_before, seed, nodes):
    n = g["n"]
    moved_in = np.bincount(after[after != before], minlength=len(w_before))
    for v in nodes:
        e = oracle.eval_node(g, phase, 0, 0, seed, bound, before, w_before, int(v))
        if not e["emit"]:
            assert after[v] == before[v], v
        elif after[v] == e["target"]:
            pass
        else:
            # rejected: with unit weights the target admitted up to its bound
            assert after[v] == before[v], v
            t = e["target"]
            assert moved_in[t] == bound - w_before[t], (v, t)
    assert len(after) == n


def test_rmat24_cluster_subround_sampled(sc, big):
    g, d = big
    n = g["n"]
    U = oracle.cluster_bound(g, 64, 18)
    col = torch.zeros(n, dtype=torch.int32, device="cuda")
    labels, rr = sc.cluster_dev(d, U, rounds=1, seed=1, level=0, color_override=col, subrounds=1)
    assert rr == 1
    after = labels.cpu().numpy()
    before = np.arange(n, dtype=np.int32)
    check_subround(g, oracle.CLUSTER, U, before, after, np.ones(n, dtype=np.int64), 1, sample_nodes(g, 3000, 1))


def test_rmat24_refine_subround_sampled(sc, big):
    g, d = big
    n, k = g["n"], 64
    Lmax = oracle.lmax(n, k, 0.03)
    before = ((np.arange(n, dtype=np.int64) * k) // n).astype(np.int32)
    part = torch.tensor(before, device="cuda")
    col = torch.zeros(n, dtype=torch.int32, device="cuda")
    sc.refine_dev(d, k, Lmax, part, rounds=1, seed=1, level=0, color_override=col, subrounds=1)
    after = part.cpu().numpy()
    w0 = np.bincount(before, minlength=k).astype(np.int64)
    check_subround(g, oracle.REFINE, Lmax, before, after, w0, 1, sample_nodes(g, 3000, 2))
    assert np.bincount(after, minlength=k).max() <= Lmax


def test_rmat24_partition_properties(sc, big):
    g, d = big
    n, k = g["n"], 64
    r1 = sc.partition_dev(d, k, 0.03, 1)
    r2 = sc.partition_dev(d, k, 0.03, 1)
    p = r1["part"].cpu().numpy()
    assert np.array_equal(p, r2["part"].cpu().numpy()) and r1["cut"] == r2["cut"]
    assert p.min() >= 0 and p.max() < k
    bw = np.bincount(p, minlength=k)
    assert np.array_equal(bw, r1["block_weights"])
    assert bw.max() <= oracle.lmax(n, k, 0.03) and r1["status"] == 0
    deg = np.diff(g["xadj"])
    src = np.repeat(np.arange(n, dtype=np.int32), deg)
    cut2 = int(np.count_nonzero(p[src] != p[g["adjncy"]]))
    assert cut2 == 2 * r1["cut"]


def test_rmat24_benchmark_call_oracle_digest(sc, big, golden_dir):
    # The benchmark's exact call (explicit unit weights, default options,
    # k = 64, eps = 0.03, seed 1) against the stored digest of the oracle's
    # whole multilevel run on this graph (tests/golden/make_oracle_digests.py).
    import hashlib
    import json
    import os
    with open(os.path.join(golden_dir, "oracle_digests.json")) as f:
        gold = json.load(f)["workloads"].get("rmat24_ef16_k64")
    if gold is None:
        pytest.skip("no stored oracle digest for the 2^24 R-MAT")
    g, _ = big
    assert hashlib.sha256(g["adjncy"].tobytes()).hexdigest() == gold["input_sha256"]
    h = dict(g)
    h["adjwgt"] = np.ones(len(g["adjncy"]), dtype=np.int32)
    h["vwgt"] = np.ones(g["n"], dtype=np.int32)
    d = sc.to_device(h, "cuda")
    part = torch.empty(g["n"], dtype=torch.int32, device="cuda")
    r = sc.partition_dev(d, 64, 0.03, 1, part=part, stream=torch.cuda.current_stream(), opts=sc.default_options())
    torch.cuda.synchronize()
    st = r["stats"]
    assert st["level_n"] == gold["level_n"] and [int(x) for x in st["level_S"]] == gold["level_S"]
    assert st["cluster_rounds"] == gold["cluster_rounds"] and st["refine_rounds"] == gold["refine_rounds"]
    assert st["visits"] == gold["visits"]
    assert r["cut"] == gold["cut"] and r["block_weights"].tolist() == gold["block_weights"]
    assert r["status"] == gold["status"]
    p = np.ascontiguousarray(part.cpu().numpy())
    assert hashlib.sha256(p.tobytes()).hexdigest() == gold["part_sha256"]
