"""Pins of the CPU oracle against values fixed outside it.

* the SplitMix64 output function against its published reference outputs;
* hand-worked examples of the update rule, the size constraint, the
  overloaded-block rule and the contraction (Section 3.1, Section 4.3);
* the balance bound Lmax = (1+eps) ceil(c(V)/k) (Section 2.1) in exact
  rational arithmetic, and the cluster bound U (Section 3.1).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def test_splitmix64_published_vectors(golden_dir):
    gold = _load(golden_dir, "splitmix64_vectors.json")
    for st in gold["streams"]:
        s = st["seed"]
        outs = st.get("outputs") or [int(h, 16) for h in st["outputs_hex"]]
        for i, expect in enumerate(outs):
            assert oracle.mix((s + i * GAMMA) & M64) == expect


def test_hash_chain_structure():
    # H of one word is mix of that word; chaining feeds the previous hash.
    for w in (0, 1, 12345, M64):
        assert oracle.hash_words([w]) == oracle.mix(w)
    a = oracle.hash_words([7, 1, 0, 0])
    b = oracle.hash_words([7, 1, 0, 1])
    assert a != b
    # colour and tie are the documented chains
    h4 = oracle.hash_words([5, 1, 3, 1, 42])
    assert oracle.color(5, 3, 1, 42, 4) == h4 % 4
    assert oracle.tie(5, 3, 1, 2, 9) == oracle.hash_words([5, 2, 3, 1, 2, 9])


def test_colors_roughly_uniform():
    cols = np.array([oracle.color(1, 0, 0, v, 4) for v in range(20000)])
    counts = np.bincount(cols, minlength=4)
    assert counts.min() > 4700 and counts.max() < 5300


def _graph(ex):
    return synth.from_edges(ex["n"], [tuple(e) for e in ex["edges"]], ex["weights"])


@pytest.mark.parametrize("name", ["A_admission_by_gain", "B_admission_by_node_id"])
def test_handworked_clustering(golden_dir, name):
    ex = _load(golden_dir, "handworked.json")[name]
    g = _graph(ex)
    lab, rr, visits = oracle.cluster(g, ex["U"], rounds=ex["rounds"], seed=ex["seed"], nsub=ex["nsub"],
                                     color_override=np.array(ex["colors"], dtype=np.int32))
    assert lab.tolist() == ex["expected_labels"]
    assert rr == ex["expected_rounds_run"]
    assert visits == rr * int(g["xadj"][-1])
    if "expected_C" in ex:
        C, cg = oracle.contract(g, lab)
        assert C.tolist() == ex["expected_C"]
        for key, val in ex["expected_coarse"].items():
            got = cg[key] if key == "n" else cg[key].tolist()
            assert got == val, key


def test_handworked_overloaded_rule(golden_dir):
    ex = _load(golden_dir, "handworked.json")["C_overloaded_rule"]
    g = _graph(ex)
    assert oracle.lmax(ex["n"], ex["k"], ex["eps"]) == ex["Lmax"]
    part, rr, _ = oracle.refine(g, ex["k"], ex["Lmax"], ex["initial_part"], rounds=ex["rounds"], seed=ex["seed"],
                                nsub=ex["nsub"], color_override=np.array(ex["colors"], dtype=np.int32))
    assert part.tolist() == ex["expected_part"]
    assert rr == ex["expected_rounds_run"]
    cut, bw = oracle.cut(g, part, ex["k"])
    assert cut == ex["expected_cut"] and bw.tolist() == ex["expected_block_weights"]


def test_handworked_contraction(golden_dir):
    ex = _load(golden_dir, "handworked.json")["D_contraction_ranks"]
    g = _graph(ex)
    C, cg = oracle.contract(g, np.array(ex["labels"], dtype=np.int32))
    assert C.tolist() == ex["expected_C"]
    for key, val in ex["expected_coarse"].items():
        got = cg[key] if key == "n" else cg[key].tolist()
        assert got == val, key


def test_handworked_two_cliques(golden_dir):
    ex = _load(golden_dir, "handworked.json")["E_two_cliques"]
    m = ex["clique"]
    edges = [(i, j) for i in range(m) for j in range(i + 1, m)]
    edges += [(m + i, m + j) for i in range(m) for j in range(i + 1, m)]
    edges.append((m - 1, m))
    g = synth.from_edges(2 * m, edges)
    r = oracle.partition(g, ex["k"], ex["eps"], ex["seed"])
    assert r["cut"] == ex["expected_cut"]
    assert sorted(r["block_weights"].tolist()) == ex["expected_block_weights"]


@pytest.mark.parametrize("cV,k,eps", [(16384, 2, 0.03), (1 << 20, 16, 0.03), (1 << 24, 64, 0.03),
                                      (4, 2, 0.0), (100, 3, 0.05), (7, 7, 0.01), (999983, 5, 0.013)])
def test_lmax_exact(cV, k, eps):
    # Section 2.1: Lmax = (1+eps) * ceil(c(V)/k); eps is a decimal with at
    # most six places, so Fraction(str(eps)) is its exact value.
    T = -(-cV // k)
    expect = int((1 + Fraction(str(eps))) * T)  # floor of a non-negative rational
    assert oracle.lmax(cV, k, eps) == expect


def test_bounds_at_benchmark_sizes():
    # U = max(max c(v), floor(c(V)/(18k))), Lmax as above, unit node weights.
    assert oracle.lmax(1 << 14, 2, 0.03) == 8437
    assert (1 << 14) // (18 * 2) == 455
    assert oracle.lmax(1 << 20, 16, 0.03) == 67502
    assert (1 << 20) // (18 * 16) == 3640
    assert oracle.lmax(1 << 24, 64, 0.03) == 270008
    assert (1 << 24) // (18 * 64) == 14563
    g = synth.ba(1 << 14, 8, seed=1)
    assert oracle.cluster_bound(g, 2) == 455


def test_cluster_bound_uses_heaviest_node():
    g = synth.from_edges(4, [(0, 1), (1, 2), (2, 3)], vwgt=[1, 1, 50, 1])
    assert oracle.cluster_bound(g, 2) == 50


def test_validation_status_codes():
    good = synth.from_edges(3, [(0, 1), (1, 2)])
    assert oracle.validate(good) == 0
    asym = dict(good)
    asym["adjwgt"] = np.array([1, 2, 1, 1], dtype=np.int32)  # w(1,0) != w(0,1)
    assert oracle.validate(asym) == -2
    loop = {"n": 2, "xadj": np.array([0, 1, 2]), "adjncy": np.array([0, 1], dtype=np.int32)}
    assert oracle.validate(loop) == -1
    zero = dict(good)
    zero["adjwgt"] = np.array([0, 0, 1, 1], dtype=np.int32)
    assert oracle.validate(zero) == -1
    big = dict(good)
    big["vwgt"] = np.array([2**31 - 1, 1, 0], dtype=np.int32)
    assert oracle.validate(big) == -3
    neg = dict(good)
    neg["vwgt"] = np.array([1, -1, 1], dtype=np.int32)
    assert oracle.validate(neg) == -1


def test_handworked_longest_prefix(golden_dir):
    ex = _load(golden_dir, "handworked.json")["F_longest_prefix"]
    g = synth.from_edges(ex["n"], [tuple(e) for e in ex["edges"]], ex["weights"], vwgt=ex["vwgt"])
    col = np.array(ex["colors"], dtype=np.int32)
    lab1, rr1, _ = oracle.cluster(g, ex["U"], rounds=1, seed=ex["seed"], nsub=ex["nsub"], color_override=col)
    assert lab1.tolist() == ex["expected_labels_after_1_round"] and rr1 == 1
    lab, rr, _ = oracle.cluster(g, ex["U"], rounds=10, seed=ex["seed"], nsub=ex["nsub"], color_override=col)
    assert lab.tolist() == ex["expected_labels"] and rr == ex["expected_rounds_run"]


def _splitmix_out(z):
    # the published SplitMix64 output function, written out for this test
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _h(words):
    h = _splitmix_out((words[0] + GAMMA) & M64)
    for w in words[1:]:
        h = _splitmix_out(((h ^ w) + GAMMA) & M64)
    return h


@pytest.mark.parametrize("seed", [1, 2, 3, 77])
@pytest.mark.parametrize("rnd", [0, 5])
def test_tie_break_prefers_smallest_priority(seed, rnd):
    # A centre whose ten leaves carry ten distinct labels, all with connection
    # 1: every label is eligible and tied, so the chosen target must be the
    # label of smallest priority H(seed, 2, level, phase, round, x) ("ties are
    # broken randomly", Section 3.1, read as a hash priority, smaller first).
    n = 11
    g = synth.from_edges(n, [(0, i) for i in range(1, n)])
    label = np.arange(n, dtype=np.int32)
    w = np.ones(n, dtype=np.int64)
    ev = oracle.eval_node(g, oracle.CLUSTER, 2, rnd, seed, 100, label, w, 0)
    expect = min(range(1, n), key=lambda x: (_h([seed, 2, 2, 0, rnd, x]), x))
    assert ev["target"] == expect and ev["emit"] == 1 and ev["gain"] == 1


def test_handworked_clustering_inside_blocks(golden_dir):
    ex = _load(golden_dir, "handworked.json")["G_cluster_within_blocks"]
    g = _graph(ex)
    col = np.array(ex["colors"], dtype=np.int32)
    blk = np.array(ex["block"], dtype=np.int32)
    lab, rr, visits = oracle.cluster(g, ex["U"], rounds=ex["rounds"], seed=ex["seed"], nsub=ex["nsub"],
                                     color_override=col, block=blk)
    assert lab.tolist() == ex["expected_labels"]
    assert rr == ex["expected_rounds_run"] and visits == ex["expected_visits"]
    free, _, fv = oracle.cluster(g, ex["U"], rounds=ex["rounds"], seed=ex["seed"], nsub=ex["nsub"],
                                 color_override=col)
    assert free.tolist() == ex["expected_labels_unrestricted"] and fv == ex["expected_visits_unrestricted"]
    C, cg = oracle.contract(g, lab)
    assert C.tolist() == ex["expected_C"]
    for key, val in ex["expected_coarse"].items():
        got = cg[key] if key == "n" else cg[key].tolist()
        assert got == val, key
    coarse_blk = np.zeros(cg["n"], dtype=np.int32)
    coarse_blk[C] = blk
    assert oracle.cut(cg, coarse_blk, 2)[0] == oracle.cut(g, blk, 2)[0] == ex["expected_coarse_cut"]


def test_handworked_degree_order(golden_dir):
    ex = _load(golden_dir, "handworked.json")["H_degree_order"]
    g = synth.from_edges(ex["n"], [tuple(e) for e in ex["edges"]])
    assert oracle.degree_colors(g, ex["nsub"]).tolist() == ex["expected_colors"]
    assert oracle.degree_colors(g, ex["nsub"], block=ex["block"]).tolist() == ex["expected_colors_within_blocks"]


def _rows_graph(n, rows, vwgt):
    """CSR with rows exactly as given (unsorted rows allowed), unit edge weights."""
    xadj = np.zeros(n + 1, dtype=np.int64)
    adj = []
    for v in range(n):
        adj += rows[v]
        xadj[v + 1] = len(adj)
    return {"n": n, "xadj": xadj, "adjncy": np.array(adj, dtype=np.int32),
            "adjwgt": np.ones(len(adj), dtype=np.int32), "vwgt": np.array(vwgt, dtype=np.int32)}


def test_handworked_initial_partition_growth(golden_dir):
    ex = _load(golden_dir, "handworked.json")["I_initial_partition_growth"]
    g = _rows_graph(ex["n"], ex["rows"], ex["vwgt"])
    assert oracle.validate(g) == 0
    assert -(-int(g["vwgt"].sum()) // ex["k"]) == ex["T"]
    assert oracle.initial_partition(g, ex["k"], ex["T"]).tolist() == ex["expected_part"]


def test_handworked_initial_lp_pool_rule(golden_dir):
    ex = _load(golden_dir, "handworked.json")["J_initial_lp_pool_rule"]
    g = synth.from_edges(ex["n"], [tuple(e) for e in ex["edges"]], ex["weights"], vwgt=ex["vwgt"])
    for v, hx in ex["seed_hashes_hex"].items():
        assert _h([ex["seed"], 5, ex["level"], int(v)]) == int(hx, 16)
    assert oracle.lmax(int(g["vwgt"].sum()), ex["k"], 0.0) == ex["Lmax"]
    part, rr, visits = oracle.initial_partition_lp(g, ex["k"], ex["T"], ex["Lmax"], seed=ex["seed"],
                                                   level=ex["level"], rounds=ex["rounds"], nsub=ex["nsub"])
    assert part.tolist() == ex["expected_part"]
    assert rr == ex["expected_rounds_run"] and visits == ex["expected_visits"]
    # with no round at all every pool node is dealt: the partition the rule avoids
    p0, rr0, _ = oracle.initial_partition_lp(g, ex["k"], ex["T"], ex["Lmax"], seed=ex["seed"], level=ex["level"],
                                             rounds=0, nsub=ex["nsub"])
    assert p0.tolist() == ex["expected_part_without_pool_offset"] and rr0 == 0


@pytest.mark.parametrize("seed", [0, 1, 7, 12345678901234567, M64])
def test_cycle_seed_independent_chain(seed):
    # V-cycle c >= 1 draws fresh colours and ties from the seed H(seed, 4, c);
    # the first cycle keeps the caller's seed
    assert oracle.cycle_seed(seed, 0) == seed
    for c in (1, 2, 3, 63):
        assert oracle.cycle_seed(seed, c) == _h([seed, 4, c])
