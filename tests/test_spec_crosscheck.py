"""Cross-coding of the oracle (Section 3.1 update rule, Section 4.3
contraction, Sections 4.4 and 4.5 multilevel loop): the plain C oracle and the
independent Python specification in ``spec_sclap.py`` must agree on random
tiny graphs, weighted and unweighted, with isolated nodes, under random
bounds, block counts and options."""
import numpy as np
import pytest

import oracle
import spec_sclap as spec
import synth


def random_graph(rng):
    n = int(rng.integers(1, 65))
    p = float(rng.choice([0.02, 0.08, 0.2, 0.5]))
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    iso = rng.random() < 0.5  # some nodes forced isolated
    if iso and n > 2:
        dead = set(rng.choice(n, size=max(1, n // 5), replace=False).tolist())
        edges = [(u, v) for u, v in edges if u not in dead and v not in dead]
    weighted = rng.random() < 0.5
    ew = rng.integers(1, 9, size=len(edges)).tolist() if weighted else None
    vw = rng.integers(0 if rng.random() < 0.2 else 1, 5, size=n).tolist() if rng.random() < 0.5 else None
    return synth.from_edges(n, edges, ew, vwgt=vw)


def node_weights(g):
    return np.ones(g["n"], dtype=np.int64) if g.get("vwgt") is None else g["vwgt"].astype(np.int64)


@pytest.mark.parametrize("block", range(10))
def test_cluster_refine_contract_agree(block):
    rng = np.random.default_rng(1000 + block)
    for _ in range(40):
        g = random_graph(rng)
        n = g["n"]
        c = node_weights(g)
        nsub = int(rng.choice([1, 2, 4, 7]))
        seed = int(rng.integers(0, 1 << 62))
        level = int(rng.integers(0, 5))
        U = int(max(c.max(initial=0), rng.integers(1, 12)))
        blk = rng.integers(0, 3, size=n).astype(np.int32) if rng.random() < 0.3 else None
        lab, rr, vis = oracle.cluster(g, U, rounds=10, seed=seed, level=level, nsub=nsub, block=blk)
        slab, srr, svis = spec.cluster(g, U, 10, seed, level, nsub, None, None if blk is None else blk.tolist())
        assert lab.tolist() == slab and rr == srr and vis == svis
        C, cg = oracle.contract(g, lab)
        sC, scg = spec.contract(g, slab)
        assert C.tolist() == sC
        for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
            assert cg[key].tolist() == scg[key], key
        k = int(rng.integers(1, 9))
        eps = float(rng.choice([0.0, 0.03, 0.2]))
        Lmax = spec.lmax(int(c.sum()), k, eps)
        assert oracle.lmax(int(c.sum()), k, eps) == Lmax
        part0 = rng.integers(0, k, size=n).astype(np.int32)
        p, prr, pvis = oracle.refine(g, k, Lmax, part0, rounds=10, seed=seed, level=level, nsub=nsub)
        sp, sprr, spvis = spec.refine(g, k, Lmax, part0.tolist(), 10, seed, level, nsub)
        assert p.tolist() == sp and prr == sprr and pvis == spvis
        assert list(oracle.cut(g, p, k)[1]) == spec.cut(g, sp, k)[1]
        assert oracle.degree_colors(g, nsub, block=blk).tolist() == spec.degree_colors(
            spec.adjacency(g)[0], nsub, None if blk is None else blk.tolist())


@pytest.mark.parametrize("block", range(10))
def test_initial_partitioners_agree(block):
    rng = np.random.default_rng(2000 + block)
    for _ in range(30):
        g = random_graph(rng)
        c = node_weights(g)
        k = int(rng.integers(1, 9))
        T = -(-int(c.sum()) // k) if c.sum() else 0
        assert oracle.initial_partition(g, k, T).tolist() == spec.initial_partition(g, k, T)
        Lmax = spec.lmax(int(c.sum()), k, 0.03)
        seed = int(rng.integers(0, 1 << 62))
        rounds = int(rng.choice([0, 1, 10]))
        nsub = int(rng.choice([1, 4]))
        p, rr, vis = oracle.initial_partition_lp(g, k, T, Lmax, seed=seed, level=1, rounds=rounds, nsub=nsub)
        sp, srr, svis = spec.initial_partition_lp(g, k, T, Lmax, seed, 1, rounds, nsub)
        assert p.tolist() == sp and rr == srr and vis == svis


@pytest.mark.parametrize("block", range(20))
def test_multilevel_partition_agrees(block):
    rng = np.random.default_rng(3000 + block)
    for _ in range(25):
        g = random_graph(rng)
        k = int(rng.integers(1, 9))
        eps = float(rng.choice([0.0, 0.01, 0.03, 0.1]))
        seed = int(rng.integers(0, 1 << 62))
        opts = dict(coarsest_nodes=int(rng.choice([1, 4, 12, 40])), subrounds=int(rng.choice([1, 2, 4])),
                    coarsen_rounds=int(rng.choice([1, 3, 10])), refine_rounds=int(rng.choice([0, 2, 10])),
                    max_levels=int(rng.choice([0, 1, 64])), vcycles=int(rng.choice([1, 1, 2, 3])),
                    degree_order=int(rng.random() < 0.3), initial=int(rng.random() < 0.3),
                    cluster_divisor=int(rng.choice([1, 18])))
        r = oracle.partition(g, k, eps, seed, **opts)
        s = spec.partition(g, k, eps, seed, **opts)
        assert r["part"].tolist() == s["part"], opts
        assert r["cut"] == s["cut"] and r["block_weights"].tolist() == s["block_weights"]
        assert r["status"] == s["status"] and r["visits"] == s["visits"]
