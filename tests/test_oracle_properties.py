"""Properties of the CPU oracle that the paper and the mathematics fix.

Each check is computed here from scratch in Python, not by calling back into
the oracle's own arithmetic:

* size constraint (Section 3.1): after every sub-round no cluster / block that
  started within the bound exceeds it; the weight array equals the weights
  recomputed from the labels;
* with a proper colouring (no two adjacent nodes share a sub-round), the cut
  of the labelling drops by exactly the sum of the gains of the moved nodes;
* convergence: when a run stops on a round without moves, no node has an
  eligible neighbouring label with a strictly larger connection, and no node of
  an overloaded block has any eligible neighbouring block;
* contraction (Section 3.1, Section 4.3): node and edge weight totals, the
  coarse graph is symmetric with sorted rows, and any coarse partition has the
  same cut and block weights as its projection (the property the paper states
  for contraction);
* special cases: U = 1 gives the identity clustering (Section 2.1), k = 1 gives
  cut 0, an edgeless graph never moves, unbounded LP on disjoint cliques
  converges to one cluster per clique;
* brute force: for n <= 16 the optimal balanced bipartition cut is a lower
  bound for the multilevel result, which must be balanced;
* storage-order independence: permuting the neighbours inside rows changes
  nothing;
* clustering inside the blocks of a partition (Section 4.4, iterated
  V-cycles): every cluster lies in one block, contracting keeps the cut and
  the block weights, one block reduces to plain clustering and singleton
  blocks to the identity; a later V-cycle equals its composition from the
  single operations.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


# ----------------------------------------------------------- python helpers

def rows(g):
    xa, adj = g["xadj"], g["adjncy"]
    ew = g.get("adjwgt")
    out = []
    for v in range(g["n"]):
        b, e = int(xa[v]), int(xa[v + 1])
        out.append([(int(adj[i]), 1 if ew is None else int(ew[i])) for i in range(b, e)])
    return out


M64 = (1 << 64) - 1


def sm_mix(z):
    """SplitMix64's published output function applied to z + golden gamma,
    written out here independently of the oracle."""
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def sm_hash(*w):
    h = sm_mix(w[0])
    for x in w[1:]:
        h = sm_mix(h ^ x)
    return h


def vw(g):
    return np.ones(g["n"], dtype=np.int64) if g.get("vwgt") is None else g["vwgt"].astype(np.int64)


def py_cut(g, lab):
    s = 0
    for v, r in enumerate(rows(g)):
        for u, w in r:
            if lab[u] != lab[v]:
                s += w
    return s // 2


def py_weights(g, lab, size):
    out = np.zeros(size, dtype=np.int64)
    np.add.at(out, np.asarray(lab, dtype=np.int64), vw(g))
    return out


def py_conns(r, lab):
    c = {}
    for u, w in r:
        c[lab[u]] = c.get(lab[u], 0) + w
    return c


def py_converged(g, lab, w, bound, refine):
    c = vw(g)
    for v, r in enumerate(rows(g)):
        if not r:
            continue
        a = lab[v]
        conn = py_conns(r, lab)
        own = conn.get(a, 0)
        elig = [x for x in conn if x != a and w[x] + c[v] <= bound]
        if refine and w[a] > bound and elig:
            return False
        if any(conn[x] > own for x in elig):
            return False
    return True


def random_graph(n, p, seed, weighted=True, node_weights=False):
    rng = np.random.default_rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    ws = rng.integers(1, 5, size=len(edges)).tolist() if weighted else None
    vwg = rng.integers(0, 4, size=n).tolist() if node_weights else None
    return synth.from_edges(n, edges, ws, vwgt=vwg)


def proper_coloring(g, ncol):
    """Greedy proper colouring with at most ncol colours, or None."""
    col = [-1] * g["n"]
    for v, r in enumerate(rows(g)):
        used = {col[u] for u, _ in r}
        free = [c for c in range(ncol) if c not in used]
        if not free:
            return None
        col[v] = free[0]
    return np.array(col, dtype=np.int32)


GRAPHS = [
    ("ba", lambda: synth.ba(300, 3, seed=4, weighted=True)),
    ("rgg", lambda: synth.rgg(400, seed=5, weighted=True)),
    ("rmat", lambda: synth.rmat(9, 8, seed=6, weighted=True)),
    ("dense_nodew", lambda: random_graph(60, 0.15, 7, node_weights=True)),
]


# ------------------------------------------------ size constraint invariants

@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("U", [1, 3, 10, 40])
def test_cluster_subround_invariants(name, make, U):
    g = make()
    n = g["n"]
    c = vw(g)
    U = max(U, int(c.max()))
    lab = np.arange(n, dtype=np.int32)
    w = c.copy()
    total = int(c.sum())
    for r in range(4):
        for s in range(4):
            oracle.subround(g, oracle.CLUSTER, 0, r, s, 4, 9, U, lab, w)
            assert w.max() <= U
            assert int(w.sum()) == total
            assert np.array_equal(w, py_weights(g, lab, n))
            assert lab.min() >= 0 and lab.max() < n


@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("k", [2, 5])
def test_refine_subround_invariants(name, make, k):
    g = make()
    n = g["n"]
    c = vw(g)
    Lmax = oracle.lmax(int(c.sum()), k, 0.03)
    rng = np.random.default_rng(3)
    part = rng.integers(0, k, size=n).astype(np.int32)
    w = py_weights(g, part, k)
    start = w.copy()
    for r in range(3):
        for s in range(4):
            oracle.subround(g, oracle.REFINE, 0, r, s, 4, 9, Lmax, part, w)
            assert np.array_equal(w, py_weights(g, part, k))
            # blocks that started within the bound stay within it
            assert all(w[b] <= Lmax for b in range(k) if start[b] <= Lmax)


@pytest.mark.parametrize("name,make", GRAPHS)
def test_gain_identity_under_proper_coloring(name, make):
    g = make()
    n = g["n"]
    col = proper_coloring(g, 64)
    assert col is not None
    ncol = int(col.max()) + 1
    c = vw(g)
    U = max(8, int(c.max()))
    lab = np.arange(n, dtype=np.int32)
    w = c.copy()
    for s in range(ncol):
        gains = {}
        for v in np.nonzero(col == s)[0]:
            ev = oracle.eval_node(g, oracle.CLUSTER, 0, 0, 9, U, lab, w, int(v))
            if ev["emit"]:
                gains[int(v)] = ev["gain"]
        before = py_cut(g, lab)
        old = lab.copy()
        oracle.subround(g, oracle.CLUSTER, 0, 0, s, ncol, 9, U, lab, w, color_override=col)
        moved = np.nonzero(lab != old)[0]
        assert all(int(v) in gains for v in moved)
        assert before - py_cut(g, lab) == sum(gains[int(v)] for v in moved)


# ------------------------------------------------------------- convergence

@pytest.mark.parametrize("name,make", GRAPHS)
def test_convergence_predicate_cluster(name, make):
    g = make()
    c = vw(g)
    U = max(12, int(c.max()))
    lab, rr, visits = oracle.cluster(g, U, rounds=60, seed=2)
    assert visits == rr * int(g["xadj"][-1])
    w = py_weights(g, lab, g["n"])
    assert w.max() <= U
    if rr < 60:  # stopped on a round without moves
        assert py_converged(g, lab, w, U, refine=False)


@pytest.mark.parametrize("name,make", GRAPHS)
def test_convergence_predicate_refine(name, make):
    g = make()
    k = 4
    Lmax = oracle.lmax(int(vw(g).sum()), k, 0.03)
    part0 = (np.arange(g["n"]) * 7 % k).astype(np.int32)
    part, rr, _ = oracle.refine(g, k, Lmax, part0, rounds=60, seed=2)
    w = py_weights(g, part, k)
    if rr < 60:
        assert py_converged(g, part, w, Lmax, refine=True)


def test_overloaded_blocks_drain():
    # Start with everything in block 0 of a path: the overloaded rule must move
    # nodes out until the block fits (each move is to a neighbouring block).
    n = 40
    g = synth.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    part0 = np.zeros(n, dtype=np.int32)
    part0[-1] = 1
    Lmax = oracle.lmax(n, 2, 0.03)
    part, rr, _ = oracle.refine(g, 2, Lmax, part0, rounds=200, seed=1)
    w = py_weights(g, part, 2)
    assert w.max() <= Lmax


# ------------------------------------------------------------- contraction

@pytest.mark.parametrize("name,make", GRAPHS)
def test_contraction_properties(name, make):
    g = make()
    n = g["n"]
    U = max(20, int(vw(g).max()))
    lab, _, _ = oracle.cluster(g, U, rounds=5, seed=3)
    C, cg = oracle.contract(g, lab)
    m = cg["n"]
    assert m == len(set(lab.tolist()))
    # ids are ranks of the used labels
    ranks = {x: i for i, x in enumerate(sorted(set(lab.tolist())))}
    assert C.tolist() == [ranks[x] for x in lab.tolist()]
    # node weights
    assert np.array_equal(cg["vwgt"].astype(np.int64), py_weights(g, C, m))
    # edge weights: plain dictionary aggregation of inter-cluster slots
    agg = {}
    intra = 0
    for v, r in enumerate(rows(g)):
        for u, w in r:
            if C[u] == C[v]:
                intra += w
            else:
                agg[(int(C[v]), int(C[u]))] = agg.get((int(C[v]), int(C[u])), 0) + w
    got = {}
    for a, r in enumerate(rows(cg)):
        nb = [u for u, _ in r]
        assert nb == sorted(nb) and len(set(nb)) == len(nb) and a not in nb
        for u, w in r:
            got[(a, u)] = w
    assert got == agg
    assert all(got[(b, a)] == w for (a, b), w in got.items())
    total = int(g["adjwgt"].sum())
    assert int(cg["adjwgt"].sum()) == total - intra
    # any coarse partition has the same cut and balance as its projection
    rng = np.random.default_rng(11)
    for k in (2, 3, 7):
        cp = rng.integers(0, k, size=m).astype(np.int32)
        fp = oracle.project(C, cp)
        assert py_cut(g, fp) == py_cut(cg, cp)
        assert np.array_equal(py_weights(g, fp, k), py_weights(cg, cp, k))


def test_cut_and_block_weights_from_scratch():
    g = random_graph(50, 0.2, 5, node_weights=True)
    rng = np.random.default_rng(0)
    part = rng.integers(0, 6, size=50).astype(np.int32)
    cut, bw = oracle.cut(g, part, 6)
    assert cut == py_cut(g, part)
    assert np.array_equal(bw, py_weights(g, part, 6))


# ----------------------------------------------------------- special cases

@pytest.mark.parametrize("name,make", GRAPHS[:3])
def test_U_one_is_identity(name, make):
    g = make()  # unit node weights
    lab, rr, _ = oracle.cluster(g, 1, rounds=10, seed=1)
    assert np.array_equal(lab, np.arange(g["n"]))
    assert rr == 1
    C, cg = oracle.contract(g, lab)
    assert cg["n"] == g["n"] and np.array_equal(cg["xadj"], g["xadj"])


def test_k_one_cut_zero():
    g = synth.ba(500, 4, seed=2, weighted=True)
    r = oracle.partition(g, 1, 0.03, 1, coarsest_nodes=50)
    assert r["cut"] == 0 and np.all(r["part"] == 0) and r["block_weights"].tolist() == [500]


def test_edgeless_graph():
    n = 37
    g = {"n": n, "xadj": np.zeros(n + 1, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32)}
    lab, rr, visits = oracle.cluster(g, 5, rounds=10, seed=1)
    assert np.array_equal(lab, np.arange(n)) and rr == 1 and visits == 0
    r = oracle.partition(g, 4, 0.0, 1, coarsest_nodes=5)
    assert r["cut"] == 0
    # isolated nodes are dealt to the lightest block in id order
    assert r["part"].tolist() == [v % 4 for v in range(n)]


def test_unbounded_lp_on_disjoint_cliques():
    # With U >= c(V) the rule is plain label propagation; in a clique a state
    # with two labels always has a node with a strictly better label, so a
    # converged run leaves exactly one label per clique.
    sizes = [5, 9, 3, 12, 7]
    edges, base = [], 0
    for s in sizes:
        edges += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
        base += s
    g = synth.from_edges(base, edges)
    lab, rr, _ = oracle.cluster(g, base, rounds=100, seed=4)
    assert rr < 100
    base = 0
    for s in sizes:
        assert len(set(lab[base:base + s].tolist())) == 1
        base += s
    assert len(set(lab.tolist())) == len(sizes)


def test_disjoint_cliques_partition_cut_zero():
    edges = [(i, j) for i in range(30) for j in range(i + 1, 30)]
    edges += [(30 + i, 30 + j) for i in range(30) for j in range(i + 1, 30)]
    g = synth.from_edges(60, edges)
    r = oracle.partition(g, 2, 0.03, 1)
    assert r["cut"] == 0 and sorted(r["block_weights"].tolist()) == [30, 30]


def test_visits_count_full_rounds():
    g = synth.rmat(10, 8, seed=2, weighted=True)
    lab, rr, visits = oracle.cluster(g, 30, rounds=3, seed=1)
    assert visits == rr * int(g["xadj"][-1])


# ------------------------------------------------------------- brute force

def brute_force_bisection(g, Lmax):
    n = g["n"]
    c = vw(g)
    us, vs, ws = [], [], []
    for v, r in enumerate(rows(g)):
        for u, w in r:
            if u > v:
                us.append(v); vs.append(u); ws.append(w)
    masks = np.arange(1 << (n - 1), dtype=np.int64)  # node n-1 fixed in block 0
    bits = (masks[:, None] >> np.arange(n)[None, :]) & 1
    w1 = bits @ c
    ok = (w1 <= Lmax) & (c.sum() - w1 <= Lmax)
    cut = ((bits[:, us] ^ bits[:, vs]) * np.array(ws)).sum(axis=1)
    return int(cut[ok].min())


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_lower_bound(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(8, 17))
    g = random_graph(n, 0.3, 100 + seed)
    Lmax = oracle.lmax(n, 2, 0.03)
    opt = brute_force_bisection(g, Lmax)
    r = oracle.partition(g, 2, 0.03, seed, coarsest_nodes=4)
    assert r["cut"] == py_cut(g, r["part"])
    assert np.array_equal(r["block_weights"], py_weights(g, r["part"], 2))
    assert r["cut"] >= opt
    if r["status"] == 0:
        assert r["block_weights"].max() <= Lmax


# ------------------------------------------------------ storage invariance

def shuffle_rows(g, seed):
    rng = np.random.default_rng(seed)
    h = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    for v in range(g["n"]):
        b, e = int(g["xadj"][v]), int(g["xadj"][v + 1])
        p = rng.permutation(e - b) + b
        h["adjncy"][b:e] = g["adjncy"][p]
        h["adjwgt"][b:e] = g["adjwgt"][p]
    return h


def test_row_order_does_not_matter():
    g = synth.rmat(11, 8, seed=8, weighted=True)
    h = shuffle_rows(g, 1)
    a = oracle.partition(g, 8, 0.03, 5, coarsest_nodes=100)
    b = oracle.partition(h, 8, 0.03, 5, coarsest_nodes=100)
    assert np.array_equal(a["part"], b["part"]) and a["cut"] == b["cut"]
    assert a["level_n"] == b["level_n"]


def test_multilevel_outputs_consistent():
    g = synth.rmat(13, 16, seed=1, weighted=False)
    r = oracle.partition(g, 16, 0.03, 1, coarsest_nodes=500)
    k = 16
    assert r["cut"] == py_cut(g, r["part"])
    bw = py_weights(g, r["part"], k)
    assert np.array_equal(bw, r["block_weights"])
    Lmax = oracle.lmax(g["n"], k, 0.03)
    assert r["status"] == (1 if bw.max() > Lmax else 0)
    assert r["levels"] >= 1
    # levels shrink, and each kept level is strictly smaller
    assert all(a > b for a, b in zip(r["level_n"], r["level_n"][1:]))
    # same inputs, same output
    r2 = oracle.partition(g, 16, 0.03, 1, coarsest_nodes=500)
    assert np.array_equal(r["part"], r2["part"])


@pytest.mark.parametrize("seed", [1, 2])
def test_stall_rule_on_mostly_isolated_graph(seed):
    # R-MAT keeps many isolated nodes, which never cluster, so coarsening
    # stalls.  A level is kept only if it is smaller than the previous one.
    # The driver continues only after a shrink of at least 5%, so every level
    # but the last was reached by such a shrink.
    g = synth.rmat(12, 4, seed=seed)
    r = oracle.partition(g, 4, 0.03, seed, coarsest_nodes=10)
    ln = r["level_n"]
    assert r["levels"] >= 1
    for a, b in zip(ln[:-2], ln[1:-1]):
        assert 20 * b <= 19 * a
    assert ln[-1] > 10  # stopped by the stall rule, not by size


# ------------------------------------------ clustering inside blocks, V-cycles
# (Section 4.4, Iterated Multilevel Schemes)

def ceil_div(a, b):
    return -(-a // b)


def py_block_conns(r, lab, blk, v):
    c = {}
    for u, w in r:
        if blk[u] == blk[v]:
            c[lab[u]] = c.get(lab[u], 0) + w
    return c


@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("nblk", [2, 5])
def test_cluster_inside_blocks_invariants(name, make, nblk):
    g = make()
    n = g["n"]
    c = vw(g)
    blk = np.random.default_rng(nblk).integers(0, nblk, size=n).astype(np.int32)
    U = max(8, int(c.max()))
    lab, rr, visits = oracle.cluster(g, U, rounds=30, seed=3, block=blk)
    # every cluster inside one block
    owner = {}
    for v in range(n):
        assert owner.setdefault(int(lab[v]), int(blk[v])) == blk[v]
    w = py_weights(g, lab, n)
    assert w.max() <= U or U < c.max()
    if rr < 30:  # converged: no node has a stronger eligible cluster of its block
        for v, r in enumerate(rows(g)):
            conn = py_block_conns(r, lab, blk, v)
            own = conn.get(int(lab[v]), 0)
            assert not any(conn[x] > own and w[x] + c[v] <= U for x in conn if x != lab[v])
    # each round looks at the same-block slots of every node
    same = sum(1 for v, r in enumerate(rows(g)) for u, _ in r if blk[u] == blk[v])
    assert visits == rr * same
    # contracting keeps every cut edge: the inherited coarse partition has
    # the cut and the block weights of the input partition
    C, cg = oracle.contract(g, lab)
    cb = np.zeros(cg["n"], dtype=np.int32)
    cb[C] = blk
    assert np.array_equal(cb[C], blk)
    assert py_cut(cg, cb) == py_cut(g, blk)
    assert np.array_equal(py_weights(cg, cb, nblk), py_weights(g, blk, nblk))


@pytest.mark.parametrize("name,make", GRAPHS)
def test_cluster_inside_one_block_is_plain_clustering(name, make):
    g = make()
    U = max(10, int(vw(g).max()))
    a = oracle.cluster(g, U, rounds=10, seed=2, block=np.zeros(g["n"], dtype=np.int32))
    b = oracle.cluster(g, U, rounds=10, seed=2)
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]


@pytest.mark.parametrize("name,make", GRAPHS)
def test_cluster_inside_singleton_blocks_is_identity(name, make):
    g = make()
    lab, rr, visits = oracle.cluster(g, 10 ** 6, rounds=10, seed=2, block=np.arange(g["n"], dtype=np.int32))
    assert np.array_equal(lab, np.arange(g["n"])) and rr == 1 and visits == 0


def test_one_vcycle_is_the_plain_multilevel_run():
    g = synth.rgg(2000, seed=3, weighted=True)
    a = oracle.partition(g, 8, 0.03, 4, coarsest_nodes=150)
    b = oracle.partition(g, 8, 0.03, 4, coarsest_nodes=150, vcycles=1)
    assert np.array_equal(a["part"], b["part"]) and a["visits"] == b["visits"]
    assert oracle.cycle_seed(4, 0) == 4 and oracle.cycle_seed(4, 1) != oracle.cycle_seed(4, 2)


def py_vcycle(g, k, eps, seed, prev, cycle, coarsest):
    """One later V-cycle composed from the oracle's single operations; the
    cycle's seed H(seed, 4, cycle) comes from the independent hash chain."""
    sd = sm_hash(seed, 4, cycle)
    cV = int(vw(g).sum())
    Lmax = oracle.lmax(cV, k, eps)
    W = cV // (18 * k)
    levels, Cs = [(g, prev)], []
    while levels[-1][0]["n"] > coarsest:
        G, blk = levels[-1]
        U = max(int(vw(G).max()), W)
        lab, _, _ = oracle.cluster(G, U, rounds=10, seed=sd, level=len(Cs), block=blk)
        C, cg = oracle.contract(G, lab)
        if cg["n"] >= G["n"]:
            break
        cb = np.zeros(cg["n"], dtype=np.int32)
        cb[C] = blk
        assert py_cut(cg, cb) == py_cut(g, prev)  # no cut edge was contracted
        Cs.append(C)
        levels.append((cg, cb))
        if 20 * cg["n"] > 19 * G["n"]:
            break
    part = levels[-1][1].copy()
    for lev in range(len(levels) - 1, -1, -1):
        if lev < len(levels) - 1:
            part = oracle.project(Cs[lev], part)
        part, _, _ = oracle.refine(levels[lev][0], k, Lmax, part, rounds=10, seed=sd, level=lev)
    return part


@pytest.mark.parametrize("make,k", [(lambda: synth.ba(3000, 4, seed=2), 4),
                                    (lambda: synth.rgg(2500, seed=6, weighted=True), 16),
                                    (lambda: synth.rmat(12, 8, seed=3), 8)])
def test_vcycles_compose_from_single_operations(make, k):
    g = make()
    r1 = oracle.partition(g, k, 0.03, 7, coarsest_nodes=200)
    r2 = oracle.partition(g, k, 0.03, 7, coarsest_nodes=200, vcycles=2)
    r3 = oracle.partition(g, k, 0.03, 7, coarsest_nodes=200, vcycles=3)
    p2 = py_vcycle(g, k, 0.03, 7, r1["part"], 1, 200)
    assert np.array_equal(p2, r2["part"])
    assert np.array_equal(py_vcycle(g, k, 0.03, 7, p2, 2, 200), r3["part"])
    for r in (r2, r3):
        assert r["cut"] == py_cut(g, r["part"])
        assert np.array_equal(r["block_weights"], py_weights(g, r["part"], k))
        assert r["status"] == (1 if r["block_weights"].max() > oracle.lmax(int(vw(g).sum()), k, 0.03) else 0)


# ------------------------------------------------- degree-ordered sub-rounds
# (Section 3.1, Section 4.1)

@pytest.mark.parametrize("name,make", GRAPHS + [("rmat_iso", lambda: synth.rmat(10, 2, seed=8))])
@pytest.mark.parametrize("nsub", [1, 2, 4, 7])
@pytest.mark.parametrize("blocked", [False, True])
def test_degree_colors_partition_by_degree(name, make, nsub, blocked):
    g = make()
    n = g["n"]
    blk = np.random.default_rng(2).integers(0, 3, size=n).astype(np.int32) if blocked else None
    col = oracle.degree_colors(g, nsub, block=blk)
    deg = np.array([sum(1 for u, _ in r if blk is None or blk[u] == blk[v]) for v, r in enumerate(rows(g))])
    pos = np.flatnonzero(deg > 0)
    assert np.all(col[deg == 0] == 0)
    cnt = len(pos)
    for s in range(nsub):
        members = pos[col[pos] == s]
        # ranks r with floor(r * nsub / cnt) == s: r in [ceil(s cnt / nsub), ceil((s+1) cnt / nsub))
        assert len(members) == ceil_div((s + 1) * cnt, nsub) - ceil_div(s * cnt, nsub)
    # every (degree, id) of a sub-round precedes every one of the next
    for s in range(nsub - 1):
        a = [(deg[v], v) for v in pos if col[v] == s]
        b = [(deg[v], v) for v in pos if col[v] == s + 1]
        if a and b:
            assert max(a) < min(b)


def py_multilevel(g, k, eps, seed, coarsest, degree_order):
    """The first multilevel cycle composed from the oracle's single operations."""
    cV = int(vw(g).sum())
    Lmax = oracle.lmax(cV, k, eps)
    W = cV // (18 * k)
    levels, Cs = [g], []
    while levels[-1]["n"] > coarsest:
        G = levels[-1]
        U = max(int(vw(G).max()), W)
        col = oracle.degree_colors(G, 4) if degree_order else None
        lab, _, _ = oracle.cluster(G, U, rounds=10, seed=seed, level=len(Cs), color_override=col)
        C, cg = oracle.contract(G, lab)
        if cg["n"] >= G["n"]:
            break
        Cs.append(C)
        levels.append(cg)
        if 20 * cg["n"] > 19 * G["n"]:
            break
    part = oracle.initial_partition(levels[-1], k, -(-cV // k))
    for lev in range(len(levels) - 1, -1, -1):
        if lev < len(levels) - 1:
            part = oracle.project(Cs[lev], part)
        part, _, _ = oracle.refine(levels[lev], k, Lmax, part, rounds=10, seed=seed, level=lev)
    return part


@pytest.mark.parametrize("make,k", [(lambda: synth.ba(3000, 4, seed=2), 4),
                                    (lambda: synth.rmat(12, 8, seed=3, weighted=True), 8)])
def test_degree_order_composes_from_single_operations(make, k):
    g = make()
    r = oracle.partition(g, k, 0.03, 5, coarsest_nodes=200, degree_order=1)
    assert np.array_equal(py_multilevel(g, k, 0.03, 5, 200, True), r["part"])
    plain = oracle.partition(g, k, 0.03, 5, coarsest_nodes=200)
    assert np.array_equal(py_multilevel(g, k, 0.03, 5, 200, False), plain["part"])
    assert r["cut"] == py_cut(g, r["part"])


# --------------------------------------- label-propagation initial partition

def test_initial_lp_edgeless_closed_form():
    # no node has neighbours: no seed, every node stays in the pool and the
    # pool fills blocks 0, 1, ... up to T in id order
    n, k = 10, 3
    g = {"n": n, "xadj": np.zeros(n + 1, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32)}
    T = -(-n // k)
    part, rr, visits = oracle.initial_partition_lp(g, k, T, oracle.lmax(n, k, 0.03), seed=3)
    assert part.tolist() == [v // T for v in range(n)] and visits == 0


@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("k", [2, 7, 32])
def test_initial_lp_properties(name, make, k):
    g = make()
    c = vw(g)
    cV = int(c.sum())
    T = -(-cV // k)
    Lmax = oracle.lmax(cV, k, 0.03)
    part, rr, _ = oracle.initial_partition_lp(g, k, T, Lmax, seed=4, level=2, rounds=10)
    assert part.min() >= 0 and part.max() < k
    bw = py_weights(g, part, k)
    assert bw.max() <= max(Lmax, T + int(c.max()) - 1)
    # with no label-propagation round every node but the seeds is dealt into
    # the remaining room: each block stays within T plus one node
    p0, rr0, v0 = oracle.initial_partition_lp(g, k, T, Lmax, seed=4, level=2, rounds=0)
    assert rr0 == 0 and v0 == 0
    assert py_weights(g, p0, k).max() <= T + int(c.max())
    # the same inputs give the same partition
    again, _, _ = oracle.initial_partition_lp(g, k, T, Lmax, seed=4, level=2, rounds=10)
    assert np.array_equal(again, part)


def test_initial_lp_seeds_are_smallest_hashes():
    # rounds = 0, unit weights: block i holds seed i, and the other nodes
    # follow in id order; the seeds are the k nodes with neighbours of
    # smallest H(seed, 5, level, v), computed here with an independent
    # SplitMix64 chain
    M64 = (1 << 64) - 1

    def mix(z):
        z = (z + 0x9E3779B97F4A7C15) & M64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)

    def H(*w):
        h = mix(w[0])
        for x in w[1:]:
            h = mix(h ^ x)
        return h

    g = synth.ba(60, 2, seed=5)
    k, seed, level = 4, 9, 1
    n = g["n"]
    T = -(-n // k)
    part, _, _ = oracle.initial_partition_lp(g, k, T, 10 ** 6, seed=seed, level=level, rounds=0)
    deg = np.diff(g["xadj"])
    order = sorted((H(seed, 5, level, v), v) for v in range(n) if deg[v] > 0)
    seeds = [v for _, v in order[:k]]
    for i, v in enumerate(seeds):
        assert part[v] == i
    rest = [v for v in range(n) if v not in seeds]
    room = [T - 1] * k  # each block holds its seed (weight 1)
    expect, b = [], 0
    for v in rest:
        while room[b] == 0:
            b += 1
        expect.append(b)
        room[b] -= 1
    assert part[rest].tolist() == expect


@pytest.mark.parametrize("make,k", [(lambda: synth.rmat(12, 8, seed=3, weighted=True), 8),
                                    (lambda: synth.ba(3000, 4, seed=2), 4)])
def test_initial_lp_in_the_multilevel_run(make, k):
    g = make()
    r = oracle.partition(g, k, 0.03, 5, coarsest_nodes=200, initial=1)
    assert r["cut"] == py_cut(g, r["part"])
    assert np.array_equal(r["block_weights"], py_weights(g, r["part"], k))
    assert r["status"] == (1 if r["block_weights"].max() > oracle.lmax(int(vw(g).sum()), k, 0.03) else 0)


# ------------------------------------------- all-cores evaluation (baseline)

@pytest.mark.parametrize("threads", [1, 3, 0])
def test_parallel_subround_equals_sequential(threads):
    # the CPU baseline's OpenMP evaluation loop: same moves, labels, weights
    # and visits as the sequential sub-round, clustering and refinement
    g = synth.rmat(12, 12, seed=31, weighted=True)
    n = g["n"]
    for phase, bound, lab0, nw in ((oracle.CLUSTER, 40, np.arange(n, dtype=np.int32), n),
                                   (oracle.REFINE, oracle.lmax(n, 8, 0.03),
                                    (np.arange(n) % 8).astype(np.int32), 8)):
        a_lab, b_lab = lab0.copy(), lab0.copy()
        wt = np.bincount(lab0, weights=vw(g), minlength=nw).astype(np.int64)
        a_w, b_w = wt.copy(), wt.copy()
        for rnd in range(3):
            for sub in range(4):
                ma, va, _ = oracle.subround(g, phase, 1, rnd, sub, 4, 9, bound, a_lab, a_w)
                mb, vb = oracle.subround_par(g, phase, 1, rnd, sub, 4, 9, bound, b_lab, b_w, threads=threads)
                assert ma == mb and va == vb
                assert np.array_equal(a_lab, b_lab) and np.array_equal(a_w, b_w)
