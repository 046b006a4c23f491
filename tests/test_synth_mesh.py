"""The mesh-type workloads of the paper's benchmark set (delX, rggX;
stand-ins generated here): structure checks of the generators.

A Delaunay triangulation of points in general position is a maximal planar
graph on its convex hull: with h hull vertices it has exactly 3n - 3 - h
edges, and it is connected.  The rggX radius 0.55 sqrt(ln n / n) gives an
expected degree of about pi 0.55^2 ln n away from the border.
"""
import math

import numpy as np

import synth


def check_csr(g):
    n, xa, adj = g["n"], g["xadj"], g["adjncy"]
    assert xa[0] == 0 and np.all(np.diff(xa) >= 0) and xa[-1] == len(adj)
    src = np.repeat(np.arange(n), np.diff(xa))
    assert np.all(src != adj), "self-loop"
    fwd = np.sort(src.astype(np.int64) * n + adj)
    bwd = np.sort(adj.astype(np.int64) * n + src)
    assert np.array_equal(fwd, bwd), "not symmetric"
    assert len(np.unique(fwd)) == len(fwd), "duplicate edge"
    return src


def connected(g):
    n, xa, adj = g["n"], g["xadj"], g["adjncy"]
    seen = np.zeros(n, dtype=bool)
    seen[0] = True
    stack = [0]
    while stack:
        u = stack.pop()
        for v in adj[xa[u]:xa[u + 1]]:
            if not seen[v]:
                seen[v] = True
                stack.append(int(v))
    return bool(seen.all())


def test_delaunay_is_a_triangulation():
    from scipy.spatial import ConvexHull
    for n, seed in ((2000, 1), (5000, 7)):
        g = synth.delaunay(n, seed=seed)
        check_csr(g)
        pts = np.random.default_rng(seed).random((n, 2))
        h = len(ConvexHull(pts).vertices)
        assert g["xadj"][-1] // 2 == 3 * n - 3 - h
        assert connected(g)
        again = synth.delaunay(n, seed=seed)
        assert np.array_equal(again["adjncy"], g["adjncy"])


def test_rgg_paper_radius_degree():
    n = 1 << 14
    g = synth.rgg_paper(n, seed=3)
    check_csr(g)
    expect = math.pi * 0.55 ** 2 * math.log(n)  # interior expectation; the border lowers it
    avg = g["xadj"][-1] / n
    assert 0.85 * expect < avg < 1.02 * expect
