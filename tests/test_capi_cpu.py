"""C-ABI checks that need no GPU.

* libsclap.so loads and exports every function include/sclap.h declares;
* the option defaults, the Lmax helper and the struct layouts match the
  header;
* the host-only routines of the library (exact validation, the initial
  partitioner) agree with the oracle's separately written ones.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1404_4797_amd as sc
    if not os.path.exists(sc.LIB_PATH):
        from paper_1404_4797_amd import build
        build.build()
    return sc, sc.load()


def _declared():
    text = open(os.path.join(ROOT, "include", "sclap.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sclap_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_calls():
    import paper_1404_4797_amd as sc
    assert _declared() == sorted(sc.EXPORTS)


def test_library_exports_every_declared_symbol():
    sc, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_options():
    sc, _ = _lib()
    o = sc.default_options()
    assert (o.coarsen_rounds, o.refine_rounds, o.subrounds, o.cluster_divisor, o.coarsest_nodes,
            o.max_levels, o.validate) == (10, 10, 4, 18, 10000, 64, 1)
    assert o.color_override is None


def test_struct_layouts_match_c(tmp_path):
    # gcc computes every field offset and struct size from the header itself
    sc, _ = _lib()
    import subprocess
    structs = {"sclap_graph": sc.Graph, "sclap_graph_owned": sc.GraphOwned, "sclap_options": sc.Options,
               "sclap_stats": sc.Stats, "sclap_batch_stats": sc.BatchStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sclap.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = dict((" ".join(l.split()[:2]), int(l.split()[2])) for l in out if l.strip())
    for cname, py in structs.items():
        assert got[cname + " size"] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[cname + " " + f] == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("cV,k,eps", [(16384, 2, 0.03), (1 << 24, 64, 0.03), (4, 2, 0.0), (999983, 5, 0.013)])
def test_lmax_matches_oracle(cV, k, eps):
    sc, _ = _lib()
    assert sc.lmax(cV, k, eps) == oracle.lmax(cV, k, eps)


def test_host_validation_matches_oracle():
    sc, _ = _lib()
    good = synth.rgg(300, seed=2, weighted=True)
    assert sc.validate(good) == 0 == oracle.validate(good)
    bad = dict(good)
    bad["adjwgt"] = good["adjwgt"].copy()
    bad["adjwgt"][5] += 1
    assert sc.validate(bad) == oracle.validate(bad) == -2
    loop = {"n": 2, "xadj": np.array([0, 1, 2]), "adjncy": np.array([0, 1], dtype=np.int32)}
    assert sc.validate(loop) == oracle.validate(loop) == -1


@pytest.mark.parametrize("make", [
    lambda: synth.rmat(11, 8, seed=4, weighted=True),
    lambda: synth.ba(3000, 3, seed=5, weighted=True),
    lambda: synth.rgg(4000, seed=6, weighted=True),
])
@pytest.mark.parametrize("k", [1, 2, 7, 64])
def test_initial_partition_cross_coded(make, k):
    sc, _ = _lib()
    g = make()
    rng = np.random.default_rng(k)
    g["vwgt"] = rng.integers(0, 5, size=g["n"]).astype(np.int32)
    T = -(-int(g["vwgt"].sum()) // k)
    a = sc.initial_partition(g, k)
    b = oracle.initial_partition(g, k, T)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("make,k", [
    (lambda: synth.rmat(10, 8, seed=9), 4),
    # dense rows: ordered through the core bitmap
    (lambda: synth.rmat(11, 48, seed=10, weighted=True), 16),
    # rows spread thinly over a wide id range: ordered by sorting
    (lambda: synth.rgg(60000, seed=11), 8),
])
def test_initial_partition_unsorted_rows(make, k):
    sc, _ = _lib()
    g = make()
    rng = np.random.default_rng(k)
    perm = rng.permutation(g["n"]).astype(np.int32)  # relabel, so rows span the id range
    if k == 8:
        x, a = g["xadj"], g["adjncy"]
        inv = np.argsort(perm)
        deg = np.diff(x)[inv]
        nx = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
        na = np.empty_like(a)
        for v in range(g["n"]):
            o = inv[v]
            na[nx[v]:nx[v + 1]] = perm[a[x[o]:x[o + 1]]]
        g = {"n": g["n"], "xadj": nx, "adjncy": na, "adjwgt": None, "vwgt": None}
    for v in range(g["n"]):
        b, e = int(g["xadj"][v]), int(g["xadj"][v + 1])
        g["adjncy"][b:e] = g["adjncy"][b:e][rng.permutation(e - b)]
    cV = g["n"] if g.get("vwgt") is None else int(np.sum(g["vwgt"]))
    T = -(-cV // k)
    assert np.array_equal(sc.initial_partition(g, k), oracle.initial_partition(g, k, T))


def test_union_builder():
    # the host-side batch builder: graph i's ids shift by the nodes before it
    sc, _ = _lib()
    import synth
    gs = [synth.ba(30, 2, seed=1, weighted=True), synth.from_edges(0, []), synth.rgg(40, seed=2)]
    u, nb = sc.union(gs)
    assert list(nb) == [0, 30, 30, 70]
    for i, g in enumerate(gs):
        lo, hi = nb[i], nb[i + 1]
        x = u["xadj"][lo:hi + 1] - u["xadj"][lo]
        assert np.array_equal(x, g["xadj"])
        a = u["adjncy"][u["xadj"][lo]:u["xadj"][hi]] - lo
        assert np.array_equal(a, g["adjncy"])
        assert np.array_equal(u["adjwgt"][u["xadj"][lo]:u["xadj"][hi]],
                              g["adjwgt"] if g.get("adjwgt") is not None else np.ones(len(a), np.int32))


@pytest.mark.parametrize("k", [3, 64])
def test_initial_partition_many_edgeless_nodes(k):
    # a small connected core among 300 000 edgeless nodes whose weights come
    # in runs (ones broken by single heavier and zero-weight nodes), so the
    # leftover nodes are dealt in many runs and the labels are written by
    # several threads; checked against the oracle
    sc, _ = _lib()
    rng = np.random.default_rng(k)
    n = 300_000
    core = np.sort(rng.choice(n, 2000, replace=False))
    edges = set()
    for i in range(len(core)):
        for j in rng.integers(0, len(core), 3):
            if j != i:
                a, b = int(core[i]), int(core[j])
                edges.add((min(a, b), max(a, b)))
    g = synth.from_edges(n, sorted(edges))
    vw = np.ones(n, dtype=np.int32)
    vw[rng.choice(n, 3000, replace=False)] = rng.integers(2, 6, 3000)
    vw[rng.choice(n, 500, replace=False)] = 0
    vw[core] = rng.integers(1, 9, len(core))
    g["vwgt"] = vw
    T = -(-int(vw.sum()) // k)
    assert np.array_equal(sc.initial_partition(g, k), oracle.initial_partition(g, k, T))


# ------------------------------------------------- serving: batch packing

def _plan(sc, reqs, free, max_batch=64, idle=True):
    n = [r[0] for r in reqs]
    S = [r[1] for r in reqs]
    fp = [64 * a + 64 * b + (4 << 20) for a, b in reqs]
    return sc.server_plan_batch(n, S, fp, free, max_batch, idle)


def test_server_packing_rule():
    sc, _ = _lib()
    small = (1000, 8000)
    # same-size requests: the prefix that fits max_batch and the budget
    assert _plan(sc, [small] * 10, 1 << 40, max_batch=4) == 4
    assert _plan(sc, [small] * 10, 1 << 40) == 10
    fp = 64 * 1000 + 64 * 8000 + (4 << 20)
    assert _plan(sc, [small] * 10, 3 * fp) == 3
    # sizes are mixed; the footprint decides
    big = (1 << 20, 16 << 20)
    assert _plan(sc, [small, small, big, small], 1 << 40) == 4
    bfp = 64 * (1 << 20) + 64 * (16 << 20) + (4 << 20)
    assert _plan(sc, [small, small, big, small], 2 * fp + bfp - 1) == 2
    # the first request is taken when nothing else runs, whatever its footprint
    assert _plan(sc, [big], 1 << 20, idle=True) == 1
    assert _plan(sc, [big], 1 << 20, idle=False) == 0
    # the union's node count stays within int32
    huge = (1 << 30, 1 << 30)
    assert _plan(sc, [huge, huge, huge], 1 << 62) == 1
    assert _plan(sc, [], 1 << 40) == 0
