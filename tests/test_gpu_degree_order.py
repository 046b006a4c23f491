"""GPU parity of degree-ordered clustering sub-rounds (Section 3.1; Section
4.1, coarsening only) against the CPU oracle, bit for bit: clustering with
the option set equals the oracle's clustering under the oracle's degree
colours (plain and inside blocks, several sub-round counts and knob sets,
graphs with isolated nodes and multi-tile rows), and full partitions, V-cycles
and batches with the option equal the oracle's.
"""
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
    c = pad
    n = pad + 1 + n_leaves + pad
    return synth.from_edges(n, [(c, v) for v in range(pad + 1, pad + 1 + n_leaves)])


GRAPHS = {
    "ba_4k": lambda: synth.ba(4000, 4, seed=11, weighted=True),
    "rgg_6k": lambda: synth.rgg(6000, seed=12, weighted=True),
    "rmat_13": lambda: synth.rmat(13, 16, seed=13, weighted=True),
    "rmat_12_iso": lambda: synth.rmat(12, 2, seed=15),
    "star_pad": lambda: star_with_isolated(9000, 700),
}

KNOBS = [dict(), dict(lane_max_degree=2, wave_max_degree=8, block_max_degree=24), dict(skip_quiet=1),
         dict(fused_eval=-1)]


def test_handworked_degree_order_on_gpu(sc, golden_dir):
    with open(os.path.join(golden_dir, "handworked.json")) as f:
        e = json.load(f)["H_degree_order"]
    g = synth.from_edges(e["n"], [tuple(x) for x in e["edges"]])
    for U in (2, 3, 7):
        lab, rr = sc.cluster_dev(dev(sc, g), U, rounds=10, seed=3, subrounds=e["nsub"], degree_order=1)
        ref, rr_ref, _ = oracle.cluster(g, U, rounds=10, seed=3, nsub=e["nsub"],
                                        color_override=np.array(e["expected_colors"], dtype=np.int32))
        assert lab.cpu().tolist() == ref.tolist() and rr == rr_ref
        blk = np.array(e["block"], dtype=np.int32)
        lab, rr = sc.cluster_dev(dev(sc, g), U, rounds=10, seed=3, subrounds=e["nsub"], degree_order=1,
                                 block=torch.tensor(blk, device="cuda"))
        ref, rr_ref, _ = oracle.cluster(g, U, rounds=10, seed=3, nsub=e["nsub"], block=blk,
                                        color_override=np.array(e["expected_colors_within_blocks"], dtype=np.int32))
        assert lab.cpu().tolist() == ref.tolist() and rr == rr_ref


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("nsub", [1, 4, 7])
@pytest.mark.parametrize("knobs", range(len(KNOBS)))
def test_cluster_degree_order_parity(sc, gname, nsub, knobs):
    g = GRAPHS[gname]()
    d = dev(sc, g)
    U = max(3, g["n"] // 300)
    say("cluster degree order", gname, nsub, KNOBS[knobs])
    lab, rr = sc.cluster_dev(d, U, rounds=6, seed=2, level=1, subrounds=nsub, degree_order=1, **KNOBS[knobs])
    ref, rr_ref, _ = oracle.cluster(g, U, rounds=6, seed=2, level=1, nsub=nsub,
                                    color_override=oracle.degree_colors(g, nsub))
    assert rr == rr_ref and np.array_equal(lab.cpu().numpy(), ref)
    blk = np.random.default_rng(nsub).integers(0, 3, size=g["n"]).astype(np.int32)
    lab, rr = sc.cluster_dev(d, U, rounds=6, seed=2, level=1, subrounds=nsub, degree_order=1,
                             block=torch.tensor(blk, device="cuda"), **KNOBS[knobs])
    ref, rr_ref, _ = oracle.cluster(g, U, rounds=6, seed=2, level=1, nsub=nsub, block=blk,
                                    color_override=oracle.degree_colors(g, nsub, block=blk))
    assert rr == rr_ref and np.array_equal(lab.cpu().numpy(), ref)


def test_color_override_wins_over_degree_order(sc):
    g = synth.ba(2000, 3, seed=4)
    col = np.random.default_rng(1).integers(0, 4, size=g["n"]).astype(np.int32)
    lab, _ = sc.cluster_dev(dev(sc, g), 20, rounds=5, seed=1, degree_order=1,
                            color_override=torch.tensor(col, device="cuda"))
    ref, _, _ = oracle.cluster(g, 20, rounds=5, seed=1, color_override=col)
    assert np.array_equal(lab.cpu().numpy(), ref)


PGRAPHS = {
    "ba_4k": lambda: synth.ba(4000, 4, seed=11, weighted=True),
    "rgg_6k": lambda: synth.rgg(6000, seed=12, weighted=True),
    "rmat_13": lambda: synth.rmat(13, 16, seed=13, weighted=True),
}


@pytest.mark.parametrize("gname", list(PGRAPHS))
@pytest.mark.parametrize("k", [2, 16])
@pytest.mark.parametrize("vcycles", [1, 2])
def test_partition_degree_order_parity(sc, gname, k, vcycles):
    g = PGRAPHS[gname]()
    say("partition degree order", gname, k, vcycles)
    r = sc.partition_dev(dev(sc, g), k, 0.03, 4, coarsest_nodes=300, degree_order=1, vcycles=vcycles)
    ref = oracle.partition(g, k, 0.03, 4, coarsest_nodes=300, degree_order=1, vcycles=vcycles)
    assert r["stats"]["level_n"] == ref["level_n"] and r["stats"]["visits"] == ref["visits"]
    assert np.array_equal(r["part"].cpu().numpy(), ref["part"])
    assert r["cut"] == ref["cut"] and np.array_equal(r["block_weights"], ref["block_weights"])


def test_batch_degree_order_matches_oracle(sc):
    gs = synth.batch_mix(10, seed=5, n_lo_log2=8, n_hi_log2=13)
    ks = [g["k"] for g in gs]
    eps = [g["eps"] for g in gs]
    seeds = [g["seed"] for g in gs]
    for vc in (1, 2):
        r = sc.partition_batch(gs, ks, eps, seeds, coarsest_nodes=400, degree_order=1, vcycles=vc)
        for i, g in enumerate(gs):
            ref = oracle.partition(g, ks[i], eps[i], seeds[i], coarsest_nodes=400, degree_order=1, vcycles=vc)
            got = r["graphs"][i]
            assert np.array_equal(got["part"], ref["part"]), (vc, i)
            assert got["cut"] == ref["cut"], (vc, i)
