"""The device initial partitioner (label propagation from hashed seeds with
a pool label) against the oracle, bit for bit: the partitioner alone
(several k, round counts, weighted graphs, isolated nodes, more blocks than
nodes with neighbours) and full partitions with initial_partitioner = 1,
the batched path, plus its range checks.
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


def with_node_weights(g, seed):
    h = dict(g)
    h["vwgt"] = np.random.default_rng(seed).integers(0, 6, size=g["n"]).astype(np.int32)
    return h


GRAPHS = {
    "ba_3k": lambda: synth.ba(3000, 3, seed=1, weighted=True),
    "rmat_12": lambda: synth.rmat(12, 8, seed=2, weighted=True),
    "rmat_12_nodew": lambda: with_node_weights(synth.rmat(12, 8, seed=3), 4),
    "rgg_4k": lambda: synth.rgg(4000, seed=5, weighted=True),
    "del_13": lambda: synth.delaunay(1 << 13, seed=6),
}


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("k", [2, 16, 300])
@pytest.mark.parametrize("rounds", [0, 3, 10])
def test_initial_partitioner_parity(sc, gname, k, rounds):
    g = GRAPHS[gname]()
    vw = np.ones(g["n"], dtype=np.int64) if g.get("vwgt") is None else g["vwgt"].astype(np.int64)
    cV = int(vw.sum())
    T = -(-cV // k)
    Lmax = oracle.lmax(cV, k, 0.03)
    say("initial", gname, k, rounds)
    part, visits = sc.initial_partition_lp_dev(sc.to_device(g, "cuda"), k, T, Lmax, seed=7, level=2, rounds=rounds)
    ref, _, ref_visits = oracle.initial_partition_lp(g, k, T, Lmax, seed=7, level=2, rounds=rounds)
    assert np.array_equal(part.cpu().numpy(), ref) and visits == ref_visits


def test_initial_partitioner_isolated_and_few_seeds(sc):
    # 5 nodes with neighbours, many isolated ones, k larger than the seeds
    edges = [(0, 1), (1, 2), (2, 3), (3, 4)]
    n = 200
    g = synth.from_edges(n, edges)
    for k in (3, 8, 64):
        T = -(-n // k)
        part, _ = sc.initial_partition_lp_dev(sc.to_device(g, "cuda"), k, T, oracle.lmax(n, k, 0.0), seed=2)
        ref, _, _ = oracle.initial_partition_lp(g, k, T, oracle.lmax(n, k, 0.0), seed=2)
        assert np.array_equal(part.cpu().numpy(), ref)


@pytest.mark.parametrize("gname", ["ba_3k", "rmat_12", "rgg_4k", "del_13"])
@pytest.mark.parametrize("k", [2, 16])
def test_partition_with_device_initial(sc, gname, k):
    g = GRAPHS[gname]()
    say("partition initial=1", gname, k)
    r = sc.partition_dev(sc.to_device(g, "cuda"), k, 0.03, 4, coarsest_nodes=300, initial_partitioner=1)
    ref = oracle.partition(g, k, 0.03, 4, coarsest_nodes=300, initial=1)
    assert r["stats"]["level_n"] == ref["level_n"] and r["stats"]["visits"] == ref["visits"]
    assert np.array_equal(r["part"].cpu().numpy(), ref["part"])
    assert r["cut"] == ref["cut"] and r["status"] == ref["status"]


def test_device_initial_range_checks(sc):
    g = synth.ba(500, 2, seed=1)
    with pytest.raises(sc.SclapError):
        sc.partition(g, 4, 0.03, 1, initial_partitioner=2)


def test_batch_with_device_initial(sc):
    # every graph of a batch gets its own seeds, pool, bound and rooms: its
    # result equals the oracle's for that graph alone
    gs = synth.batch_mix(12, seed=8, n_lo_log2=8, n_hi_log2=13)
    ks = [g["k"] for g in gs]
    eps = [g["eps"] for g in gs]
    seeds = [g["seed"] for g in gs]
    for vc in (1, 2):
        say("batch initial=1 vcycles", vc)
        r = sc.partition_batch(gs, ks, eps, seeds, coarsest_nodes=400, initial_partitioner=1, vcycles=vc)
        for i, g in enumerate(gs):
            ref = oracle.partition(g, ks[i], eps[i], seeds[i], coarsest_nodes=400, initial=1, vcycles=vc)
            got = r["graphs"][i]
            assert np.array_equal(got["part"], ref["part"]), (vc, i)
            assert got["cut"] == ref["cut"], (vc, i)
