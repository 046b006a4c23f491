"""Seeded synthetic graph generators (inputs only).

Stand-ins for the paper's benchmark graphs (Section 5, Table I), which are not
available here.  This module draws random graphs and assembles symmetric CSR
arrays; it contains none of the partitioning method's arithmetic.  The CPU
oracle and the GPU library both consume its output and share no other code.

Every function returns a dict with numpy arrays::

    {"n": int, "xadj": int64[n+1], "adjncy": int32[S], "adjwgt": int32[S],
     "vwgt": int32[n]}

Rows are sorted ascending, symmetric, without self-loops or duplicates.
Random draws come from a counter-based SplitMix64 stream (Steele, Lea, Flood,
OOPSLA 2014) addressed by index, so the output is independent of thread count.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force=False):
    """Compile libsynth.so with gcc (OpenMP for the parallel loops)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P64 = ctypes.POINTER(ctypes.c_int64)
        PP32 = ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))
        lib.synth_rmat.restype = ctypes.c_int64
        lib.synth_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                   P64, PP32, PP32]
        lib.synth_ba.restype = ctypes.c_int64
        lib.synth_ba.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                                 P64, PP32, PP32]
        lib.synth_rgg.restype = ctypes.c_int64
        lib.synth_rgg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                  P64, PP32, PP32]
        lib.synth_take_i32.restype = None
        lib.synth_take_i32.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_int64]
        lib.synth_draw.restype = ctypes.c_uint64
        lib.synth_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


def _finish(n, S, xadj, padj, pw):
    lib = _load()
    adj = np.empty(S, dtype=np.int32)
    w = np.empty(S, dtype=np.int32)
    lib.synth_take_i32(padj, adj.ctypes.data, S)
    lib.synth_take_i32(pw, w.ctypes.data, S)
    return {"n": int(n), "xadj": xadj, "adjncy": adj, "adjwgt": w,
            "vwgt": np.ones(n, dtype=np.int32)}


def _outs(n):
    xadj = np.zeros(n + 1, dtype=np.int64)
    padj = ctypes.POINTER(ctypes.c_int32)()
    pw = ctypes.POINTER(ctypes.c_int32)()
    return xadj, padj, pw


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=1, weighted=False, n=None):
    """R-MAT graph with ``edge_factor * 2**scale`` draws, no noise, no permutation.

    ``n`` (default ``2**scale``) keeps only nodes ``< n``; draws touching other
    nodes are dropped.
    """
    nk = (1 << scale) if n is None else int(n)
    ne = int(edge_factor) * (1 << scale)
    xadj, padj, pw = _outs(nk)
    S = _load().synth_rmat(scale, nk, ne, a, b, c, seed, int(bool(weighted)),
                           xadj.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           ctypes.byref(padj), ctypes.byref(pw))
    return _finish(nk, S, xadj, padj, pw)


def ba(n, m=8, seed=1, weighted=False):
    """Barabasi-Albert graph: nodes 0..m-1 unconnected, node m joins all of them,
    later nodes attach to m distinct degree-proportional targets."""
    xadj, padj, pw = _outs(n)
    S = _load().synth_ba(n, m, seed, int(bool(weighted)),
                         xadj.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         ctypes.byref(padj), ctypes.byref(pw))
    return _finish(n, S, xadj, padj, pw)


def rgg(n, radius=None, seed=1, weighted=False):
    """2D random geometric graph on the unit square.

    The default radius sqrt(8/(pi n)) gives an average degree near 8.
    """
    if radius is None:
        radius = math.sqrt(8.0 / (math.pi * max(n, 1)))
    xadj, padj, pw = _outs(n)
    S = _load().synth_rgg(n, radius, seed, int(bool(weighted)),
                          xadj.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          ctypes.byref(padj), ctypes.byref(pw))
    return _finish(n, S, xadj, padj, pw)


def rgg_paper(n, seed=1, weighted=False):
    """rggX of the paper's benchmark set: radius 0.55 sqrt(ln n / n), chosen
    there so that the graph is almost surely connected."""
    return rgg(n, radius=0.55 * math.sqrt(math.log(max(n, 2)) / max(n, 1)), seed=seed, weighted=weighted)


def delaunay(n, seed=1):
    """delX of the paper's benchmark set: the Delaunay triangulation of n
    points drawn uniformly from the unit square (numpy generator seeded with
    ``seed``; triangulation by scipy's Qhull).  Unit weights, sorted rows."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    key = np.unique(e[:, 0] * n + e[:, 1])
    u, v = key // n, key % n
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.argsort(src * n + dst, kind="stable")
    src, dst = src[order], dst[order]
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.add.at(xadj, src + 1, 1)
    xadj = np.cumsum(xadj)
    return {"n": n, "xadj": xadj, "adjncy": dst.astype(np.int32), "adjwgt": None, "vwgt": None}


def draw(key, i):
    """i-th output of the SplitMix64 stream seeded with ``key``."""
    return int(_load().synth_draw(key, i))


def from_edges(n, edges, weights=None, vwgt=None):
    """Symmetric CSR from an undirected edge list (tiny hand-made graphs).

    ``edges`` is a list of (u, v); ``weights`` an optional list of the same
    length.  Rows come out sorted.  Duplicate pairs are merged keeping the
    first weight.
    """
    adj = [dict() for _ in range(n)]
    for i, (u, v) in enumerate(edges):
        if u == v:
            raise ValueError("self-loop")
        w = 1 if weights is None else int(weights[i])
        adj[u].setdefault(v, w)
        adj[v].setdefault(u, w)
    xadj = np.zeros(n + 1, dtype=np.int64)
    cols, ws = [], []
    for u in range(n):
        for v in sorted(adj[u]):
            cols.append(v)
            ws.append(adj[u][v])
        xadj[u + 1] = len(cols)
    return {"n": n, "xadj": xadj, "adjncy": np.array(cols, dtype=np.int32),
            "adjwgt": np.array(ws, dtype=np.int32),
            "vwgt": (np.ones(n, dtype=np.int32) if vwgt is None else np.asarray(vwgt, dtype=np.int32))}


def batch_mix(count=512, seed=0, n_lo_log2=10, n_hi_log2=18, progress=None):
    """Mixed batch of graphs: a third each of BA, R-MAT and 2D RGG.

    Graph i: n = round(2**(lo + (hi-lo)*u)) with u uniform in [0,1);
    type i mod 3: BA with m in {4, 8, 16}; R-MAT with edge factor in [8, 16]
    (drawn at scale ceil(log2 n), ids >= n dropped); RGG with average degree
    near 8.  Edge weights uniform in [1, 4].  k is a power of two in [2, 64],
    eps in {0.01, 0.03, 0.05}, seed 1000 + i.
    Returns a list of dicts (graph arrays plus "k", "eps", "seed", "kind").
    ``progress(i)``, if given, is called after every 100th graph.
    """
    key = (seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF
    out = []
    for i in range(count):
        r0 = draw(key, 4 * i)
        r1 = draw(key, 4 * i + 1)
        r2 = draw(key, 4 * i + 2)
        u = (r0 >> 11) / float(1 << 53)
        n = int(round(2.0 ** (n_lo_log2 + (n_hi_log2 - n_lo_log2) * u)))
        gseed = 1000 + i
        kind = i % 3
        if kind == 0:
            m = (4, 8, 16)[r1 % 3]
            g = ba(n, m, seed=gseed, weighted=True)
            g["kind"] = "ba%d" % m
        elif kind == 1:
            ef = 8 + int(r1 % 9)
            sc = max(1, int(math.ceil(math.log2(n))))
            g = rmat(sc, edge_factor=ef, seed=gseed, weighted=True, n=n)
            g["kind"] = "rmat%d" % ef
        else:
            g = rgg(n, seed=gseed, weighted=True)
            g["kind"] = "rgg"
        g["k"] = 2 << int(r2 % 6)
        g["eps"] = (0.01, 0.03, 0.05)[(r2 >> 8) % 3]
        g["seed"] = gseed
        out.append(g)
        if progress is not None and (i + 1) % 100 == 0:
            progress(i + 1)
    return out
