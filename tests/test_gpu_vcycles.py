"""GPU parity of clustering inside the blocks of a partition and of iterated
V-cycles (Section 4.4, Iterated Multilevel Schemes) against the CPU oracle,
bit for bit: labels and round counts of the restricted clustering (every
degree bucket, rows spanning several slot tiles, empty rows at the ends,
one block, singleton blocks), full partitions with 2 and 3 cycles (parts,
cuts, block weights, per-level statistics, visits), the host and batched
entry points, the option's range check, and the R-MAT scale-20 workload
against the stored digest of the oracle's output.
"""
import hashlib
import json
import os

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


def dev(sc, g):
    return sc.to_device(g, "cuda")


def star_with_isolated(n_leaves, pad):
    # pad isolated nodes, the star's centre, pad isolated nodes, the leaves,
    # pad isolated nodes: the centre's row spans several slot tiles and empty
    # rows sit at both ends and next to it
    c = pad
    leaves = list(range(pad + 1, pad + 1 + n_leaves))
    n = pad + 1 + n_leaves + pad
    return synth.from_edges(n, [(c, v) for v in leaves])


GRAPHS = {
    "ba_4k": lambda: synth.ba(4000, 4, seed=11, weighted=True),
    "rgg_6k": lambda: synth.rgg(6000, seed=12, weighted=True),
    "rmat_13": lambda: synth.rmat(13, 16, seed=13, weighted=True),
    "star_pad": lambda: star_with_isolated(9000, 700),
}

KNOBS = [dict(), dict(lane_max_degree=2, wave_max_degree=8, block_max_degree=24),
         dict(lane_max_degree=2, wave_max_degree=8, block_max_degree=40, hub_region_cap=3), dict(skip_quiet=1)]


def blocks(g, kind):
    n = g["n"]
    if kind == "random3":
        return np.random.default_rng(3).integers(0, 3, size=n).astype(np.int32)
    if kind == "ranges":  # contiguous id ranges: long runs of kept and cut slots
        return ((np.arange(n, dtype=np.int64) * 5) // max(n, 1)).astype(np.int32)
    if kind == "one":
        return np.full(n, 7, dtype=np.int32)
    if kind == "singletons":
        return np.arange(n, dtype=np.int32)
    raise ValueError(kind)


def test_handworked_inside_blocks_on_gpu(sc, golden_dir):
    with open(os.path.join(golden_dir, "handworked.json")) as f:
        e = json.load(f)["G_cluster_within_blocks"]
    g = synth.from_edges(e["n"], [tuple(x) for x in e["edges"]], e["weights"])
    col = torch.tensor(e["colors"], dtype=torch.int32, device="cuda")
    blk = torch.tensor(e["block"], dtype=torch.int32, device="cuda")
    lab, rr = sc.cluster_dev(dev(sc, g), e["U"], rounds=e["rounds"], seed=e["seed"], color_override=col,
                             subrounds=e["nsub"], block=blk)
    assert lab.cpu().tolist() == e["expected_labels"] and rr == e["expected_rounds_run"]
    lab, rr = sc.cluster(g, e["U"], rounds=e["rounds"], seed=e["seed"], color_override=np.array(e["colors"]),
                         subrounds=e["nsub"], block=np.array(e["block"]))
    assert lab.tolist() == e["expected_labels"]


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("kind", ["random3", "ranges", "one", "singletons"])
@pytest.mark.parametrize("knobs", range(len(KNOBS)))
def test_cluster_within_parity(sc, gname, kind, knobs):
    g = GRAPHS[gname]()
    d = dev(sc, g)
    blk = blocks(g, kind)
    tb = torch.tensor(blk, device="cuda")
    U = max(3, g["n"] // 300)
    for seed, nsub in ((1, 4), (6, 2)):
        say("cluster_within", gname, kind, KNOBS[knobs], "U=%d seed=%d" % (U, seed))
        lab, rr = sc.cluster_dev(d, U, rounds=6, seed=seed, level=1, subrounds=nsub, block=tb, **KNOBS[knobs])
        ref, rr_ref, _ = oracle.cluster(g, U, rounds=6, seed=seed, level=1, nsub=nsub, block=blk)
        assert rr == rr_ref
        assert np.array_equal(lab.cpu().numpy(), ref)


def test_cluster_within_on_partition_blocks(sc):
    g = synth.rmat(14, 16, seed=2, weighted=True)
    p = oracle.partition(g, 8, 0.03, 3, coarsest_nodes=500)["part"]
    U = oracle.cluster_bound(g, 8, 18)
    lab, rr = sc.cluster_dev(dev(sc, g), U, rounds=10, seed=2, block=torch.tensor(p, device="cuda"))
    ref, rr_ref, _ = oracle.cluster(g, U, rounds=10, seed=2, block=p)
    assert rr == rr_ref and np.array_equal(lab.cpu().numpy(), ref)


def test_cluster_within_empty_graphs(sc):
    e = {"n": 0, "xadj": np.zeros(1, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32)}
    lab, rr = sc.cluster(e, 5, rounds=3, block=np.zeros(0, dtype=np.int32))
    assert len(lab) == 0
    g = {"n": 40, "xadj": np.zeros(41, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32)}
    lab, rr = sc.cluster_dev(dev(sc, g), 5, rounds=3, block=torch.zeros(40, dtype=torch.int32, device="cuda"))
    assert lab.cpu().tolist() == list(range(40)) and rr == 1


PGRAPHS = {
    "ba_4k": lambda: synth.ba(4000, 4, seed=11, weighted=True),
    "rgg_6k": lambda: synth.rgg(6000, seed=12, weighted=True),
    "rmat_13": lambda: synth.rmat(13, 16, seed=13, weighted=True),
    "rmat_12_nodew": lambda: dict(synth.rmat(12, 8, seed=14, weighted=True),
                                  vwgt=np.random.default_rng(1).integers(0, 6, size=1 << 12).astype(np.int32)),
}


@pytest.mark.parametrize("gname", list(PGRAPHS))
@pytest.mark.parametrize("k", [2, 16])
@pytest.mark.parametrize("vcycles", [2, 3])
def test_partition_vcycles_parity(sc, gname, k, vcycles):
    g = PGRAPHS[gname]()
    say("partition", gname, "k=%d vcycles=%d" % (k, vcycles))
    r = sc.partition_dev(dev(sc, g), k, 0.03, 4, coarsest_nodes=300, vcycles=vcycles)
    ref = oracle.partition(g, k, 0.03, 4, coarsest_nodes=300, vcycles=vcycles)
    assert r["stats"]["level_n"] == ref["level_n"]
    assert r["stats"]["cluster_rounds"] == ref["cluster_rounds"]
    assert r["stats"]["refine_rounds"] == ref["refine_rounds"]
    assert r["stats"]["visits"] == ref["visits"]
    assert np.array_equal(r["part"].cpu().numpy(), ref["part"])
    assert r["cut"] == ref["cut"] and np.array_equal(r["block_weights"], ref["block_weights"])
    assert r["status"] == ref["status"]


def test_vcycles_host_entry_and_options(sc):
    g = synth.rmat(12, 16, seed=21, weighted=True)
    r = sc.partition(g, 8, 0.05, 2, coarsest_nodes=500, vcycles=2)
    ref = oracle.partition(g, 8, 0.05, 2, coarsest_nodes=500, vcycles=2)
    assert np.array_equal(r["part"], ref["part"]) and r["cut"] == ref["cut"]
    # 0 counts as one cycle; more than 64 is refused
    a = sc.partition(g, 8, 0.05, 2, coarsest_nodes=500, vcycles=0)
    b = oracle.partition(g, 8, 0.05, 2, coarsest_nodes=500)
    assert np.array_equal(a["part"], b["part"])
    with pytest.raises(sc.SclapError) as e:
        sc.partition(g, 8, 0.05, 2, vcycles=65)
    assert e.value.status == sc.ERR_INVALID


def test_vcycles_small_graphs_without_coarsening(sc):
    # graphs at or below coarsest_nodes: every cycle refines the previous
    # result on the input graph with the cycle's own seed
    for g, k in ((synth.ba(200, 3, seed=5), 4), (synth.rgg(300, seed=6, weighted=True), 3)):
        r = sc.partition_dev(dev(sc, g), k, 0.03, 9, vcycles=3)
        ref = oracle.partition(g, k, 0.03, 9, vcycles=3)
        assert np.array_equal(r["part"].cpu().numpy(), ref["part"]) and r["cut"] == ref["cut"]


def test_batch_vcycles_matches_oracle(sc):
    gs = synth.batch_mix(10, seed=4, n_lo_log2=8, n_hi_log2=13)
    ks = [g["k"] for g in gs]
    eps = [g["eps"] for g in gs]
    seeds = [g["seed"] for g in gs]
    say("batch vcycles", [g["n"] for g in gs])
    r = sc.partition_batch(gs, ks, eps, seeds, coarsest_nodes=400, vcycles=2)
    for i, g in enumerate(gs):
        ref = oracle.partition(g, ks[i], eps[i], seeds[i], coarsest_nodes=400, vcycles=2)
        got = r["graphs"][i]
        assert np.array_equal(got["part"], ref["part"]), i
        assert got["cut"] == ref["cut"] and np.array_equal(got["block_weights"], ref["block_weights"]), i


def test_rmat20_vcycles_digest(sc, golden_dir):
    # R-MAT scale 20, k = 16, two cycles: compared with the stored digest of
    # the oracle's output (tests/golden/make_oracle_digests.py)
    with open(os.path.join(golden_dir, "oracle_digests.json")) as f:
        w = json.load(f)["workloads"]["rmat20_ef16_k16_vcycles2"]
    g = synth.rmat(20, 16, seed=1)
    assert hashlib.sha256(g["adjncy"].tobytes()).hexdigest() == w["input_sha256"]
    r = sc.partition_dev(dev(sc, g), w["k"], w["eps"], w["seed"], **w["opts"])
    part = r["part"].cpu().numpy().astype(np.int32)
    assert r["stats"]["level_n"] == w["level_n"]
    assert r["cut"] == w["cut"] and r["block_weights"].tolist() == w["block_weights"]
    assert hashlib.sha256(part.tobytes()).hexdigest() == w["part_sha256"]
    assert r["stats"]["visits"] == w["visits"]
