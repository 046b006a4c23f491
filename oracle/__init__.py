"""Python access to the CPU oracle (``sclap_oracle.c``).

TEST INFRASTRUCTURE ONLY: the plain single-threaded reference implementation
of SCLaP, cluster contraction and the multilevel partitioner that the GPU
library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this module.  It shares no code with the
GPU library.

Graphs are dicts of numpy arrays as produced by :mod:`synth`
(``n``, ``xadj`` int64, ``adjncy`` int32, optional ``adjwgt``/``vwgt`` int32).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sclap_oracle.c")
_HDR = os.path.join(_HERE, "sclap_oracle.h")
_LIB = os.path.join(_HERE, "libsclap_oracle.so")
_lib = None

CLUSTER, REFINE = 0, 1


def build(force=False):
    """Compile the oracle with gcc (plain C, single thread)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xadj", ctypes.c_void_p), ("adjncy", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("adjwgt", ctypes.c_void_p)]


class _Eval(ctypes.Structure):
    _fields_ = [("emit", ctypes.c_int32), ("target", ctypes.c_int32), ("gain", ctypes.c_int64),
                ("conn_target", ctypes.c_int64), ("conn_own", ctypes.c_int64), ("over", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("coarsen_rounds", ctypes.c_int32), ("refine_rounds", ctypes.c_int32),
                ("subrounds", ctypes.c_int32), ("cluster_divisor", ctypes.c_int32),
                ("coarsest_nodes", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("vcycles", ctypes.c_int32), ("degree_order", ctypes.c_int32), ("initial", ctypes.c_int32)]


_MAXL = 64


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("visits", ctypes.c_int64),
                ("level_n", ctypes.c_int32 * (_MAXL + 1)), ("level_S", ctypes.c_int64 * (_MAXL + 1)),
                ("cluster_rounds", ctypes.c_int32 * (_MAXL + 1)),
                ("refine_rounds", ctypes.c_int32 * (_MAXL + 1))]


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        G = ctypes.POINTER(_Graph)
        sig = {
            "orc_mix": (u64, [u64]),
            "orc_hash": (u64, [vp, i32]),
            "orc_color": (i32, [u64, i32, i32, i32, i32]),
            "orc_tie": (u64, [u64, i32, i32, i32, i32]),
            "orc_lmax": (i64, [i64, i32, dbl]),
            "orc_cluster_bound": (i64, [G, i32, i32]),
            "orc_validate": (i32, [G]),
            "orc_eval_node": (i32, [G, i32, i32, i32, u64, i64, vp, vp, i32, ctypes.POINTER(_Eval)]),
            "orc_subround": (i64, [G, i32, i32, i32, i32, i32, u64, i64, vp, vp, vp, vp, vp]),
            "orc_cluster": (i32, [G, i64, i32, i32, u64, i32, vp, vp, vp, vp]),
            "orc_eval_node_within": (i32, [G, vp, i32, i32, i32, u64, i64, vp, vp, i32, ctypes.POINTER(_Eval)]),
            "orc_subround_within": (i64, [G, vp, i32, i32, i32, i32, i32, u64, i64, vp, vp, vp, vp, vp]),
            "orc_subround_par": (i64, [G, i32, i32, i32, i32, i32, u64, i64, vp, vp, vp, i32]),
            "orc_max_threads": (i32, []),
            "orc_cluster_within": (i32, [G, vp, i64, i32, i32, u64, i32, vp, vp, vp, vp]),
            "orc_cycle_seed": (u64, [u64, i32]),
            "orc_degree_colors": (None, [G, vp, i32, vp]),
            "orc_initial_partition_lp": (i32, [G, i32, i64, i64, u64, i32, i32, i32, vp, vp, vp]),
            "orc_refine": (i32, [G, i32, i64, i32, i32, u64, i32, vp, vp, vp, vp]),
            "orc_contract": (i32, [G, vp, vp, vp, vp, vp, vp, vp, vp]),
            "orc_project": (None, [i32, vp, vp, vp]),
            "orc_cut": (i32, [G, vp, i32, vp, vp]),
            "orc_initial_partition": (i32, [G, i32, i64, vp]),
            "orc_default_options": (None, [ctypes.POINTER(Options)]),
            "orc_partition": (i32, [G, i32, dbl, u64, ctypes.POINTER(Options), vp, vp, vp,
                                    ctypes.POINTER(_Stats)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _GraphView:
    """Keeps contiguous copies alive while the C side reads them."""

    def __init__(self, g):
        self.n = int(g["n"])
        self.xadj = np.ascontiguousarray(g["xadj"], dtype=np.int64)
        self.adjncy = np.ascontiguousarray(g["adjncy"], dtype=np.int32)
        self.vwgt = None if g.get("vwgt") is None else np.ascontiguousarray(g["vwgt"], dtype=np.int32)
        self.adjwgt = None if g.get("adjwgt") is None else np.ascontiguousarray(g["adjwgt"], dtype=np.int32)
        self.s = _Graph(self.n, _ptr(self.xadj), _ptr(self.adjncy), _ptr(self.vwgt), _ptr(self.adjwgt))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def mix(z):
    return int(_load().orc_mix(z & 0xFFFFFFFFFFFFFFFF))


def hash_words(words):
    a = np.array([w & 0xFFFFFFFFFFFFFFFF for w in words], dtype=np.uint64)
    return int(_load().orc_hash(a.ctypes.data, len(a)))


def color(seed, level, phase, v, nsub=4):
    return int(_load().orc_color(seed, level, phase, v, nsub))


def tie(seed, level, phase, rnd, x):
    return int(_load().orc_tie(seed, level, phase, rnd, x))


def lmax(cV, k, eps):
    return int(_load().orc_lmax(cV, k, eps))


def cluster_bound(g, k, divisor=18):
    gv = _GraphView(g)
    return int(_load().orc_cluster_bound(gv.ref, k, divisor))


def validate(g):
    gv = _GraphView(g)
    return int(_load().orc_validate(gv.ref))


def _block(block):
    return None if block is None else np.ascontiguousarray(block, dtype=np.int32)


def degree_colors(g, nsub=4, block=None):
    """Sub-round of every node when clustering visits nodes by increasing
    degree (Section 3.1, Section 4.1)."""
    gv = _GraphView(g)
    blk = _block(block)
    col = np.empty(gv.n, dtype=np.int32)
    _load().orc_degree_colors(gv.ref, _ptr(blk), nsub, col.ctypes.data)
    return col


def cycle_seed(seed, cycle):
    return int(_load().orc_cycle_seed(seed, cycle))


def eval_node(g, phase, level, rnd, seed, bound, label, w, v, block=None):
    gv = _GraphView(g)
    label = np.ascontiguousarray(label, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.int64)
    blk = _block(block)
    e = _Eval()
    _load().orc_eval_node_within(gv.ref, _ptr(blk), phase, level, rnd, seed, bound, label.ctypes.data,
                                 w.ctypes.data, v, ctypes.byref(e))
    return {"emit": e.emit, "target": e.target, "gain": e.gain, "conn_target": e.conn_target,
            "conn_own": e.conn_own, "over": e.over}


def subround(g, phase, level, rnd, sub, nsub, seed, bound, label, w, color_override=None, block=None):
    """One sub-round in place on ``label`` (int32) and ``w`` (int64); with
    ``block``, only same-block neighbours count.

    Returns (moves, visits, candidates)."""
    gv = _GraphView(g)
    assert label.dtype == np.int32 and w.dtype == np.int64 and label.flags.c_contiguous and w.flags.c_contiguous
    co = None if color_override is None else np.ascontiguousarray(color_override, dtype=np.int32)
    visits = np.zeros(1, dtype=np.int64)
    ncand = np.zeros(1, dtype=np.int64)
    blk = _block(block)
    moves = _load().orc_subround_within(gv.ref, _ptr(blk), phase, level, rnd, sub, nsub, seed, bound, _ptr(co),
                                        label.ctypes.data, w.ctypes.data, visits.ctypes.data,
                                        ncand.ctypes.data)
    return int(moves), int(visits[0]), int(ncand[0])


def subround_par(g, phase, level, rnd, sub, nsub, seed, bound, label, w, threads=0):
    """orc_subround with the node evaluation on ``threads`` OpenMP threads
    (0: all); in place on ``label`` and ``w``.  Returns (moves, visits)."""
    gv = _GraphView(g)
    assert label.dtype == np.int32 and w.dtype == np.int64 and label.flags.c_contiguous and w.flags.c_contiguous
    visits = np.zeros(1, dtype=np.int64)
    t = threads if threads > 0 else max_threads()
    moves = _load().orc_subround_par(gv.ref, phase, level, rnd, sub, nsub, seed, bound, label.ctypes.data,
                                     w.ctypes.data, visits.ctypes.data, t)
    return int(moves), int(visits[0])


def max_threads():
    return int(_load().orc_max_threads())


def cluster(g, U, rounds=10, seed=1, level=0, nsub=4, color_override=None, block=None):
    """Returns (labels, rounds_run, visits).  With ``block`` (int32[n]) every
    cluster stays inside one block (clustering for iterated V-cycles)."""
    gv = _GraphView(g)
    labels = np.empty(gv.n, dtype=np.int32)
    rr = np.zeros(1, dtype=np.int32)
    visits = np.zeros(1, dtype=np.int64)
    co = None if color_override is None else np.ascontiguousarray(color_override, dtype=np.int32)
    blk = _block(block)
    st = _load().orc_cluster_within(gv.ref, _ptr(blk), U, rounds, nsub, seed, level, _ptr(co), labels.ctypes.data,
                                    rr.ctypes.data, visits.ctypes.data)
    if st != 0:
        raise ValueError("orc_cluster status %d" % st)
    return labels, int(rr[0]), int(visits[0])


def refine(g, k, Lmax, part, rounds=10, seed=1, level=0, nsub=4, color_override=None):
    """Returns (part, rounds_run, visits); ``part`` is copied, not modified."""
    gv = _GraphView(g)
    p = np.array(part, dtype=np.int32, copy=True)
    rr = np.zeros(1, dtype=np.int32)
    visits = np.zeros(1, dtype=np.int64)
    co = None if color_override is None else np.ascontiguousarray(color_override, dtype=np.int32)
    st = _load().orc_refine(gv.ref, k, Lmax, rounds, nsub, seed, level, _ptr(co), p.ctypes.data,
                            rr.ctypes.data, visits.ctypes.data)
    if st != 0:
        raise ValueError("orc_refine status %d" % st)
    return p, int(rr[0]), int(visits[0])


def contract(g, labels):
    """Returns (C, coarse graph dict)."""
    gv = _GraphView(g)
    n = gv.n
    S = int(gv.xadj[n]) if n > 0 else 0
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    C = np.empty(n, dtype=np.int32)
    nc = np.zeros(1, dtype=np.int32)
    cx = np.zeros(n + 1, dtype=np.int64)
    ca = np.empty(max(S, 1), dtype=np.int32)
    cw = np.empty(max(S, 1), dtype=np.int32)
    cv = np.empty(max(n, 1), dtype=np.int32)
    Sc = np.zeros(1, dtype=np.int64)
    st = _load().orc_contract(gv.ref, labels.ctypes.data, C.ctypes.data, nc.ctypes.data, cx.ctypes.data,
                              ca.ctypes.data, cw.ctypes.data, cv.ctypes.data, Sc.ctypes.data)
    if st != 0:
        raise ValueError("orc_contract status %d" % st)
    m, s = int(nc[0]), int(Sc[0])
    return C, {"n": m, "xadj": cx[:m + 1].copy(), "adjncy": ca[:s].copy(), "adjwgt": cw[:s].copy(),
               "vwgt": cv[:m].copy()}


def project(C, coarse_part):
    C = np.ascontiguousarray(C, dtype=np.int32)
    cp = np.ascontiguousarray(coarse_part, dtype=np.int32)
    out = np.empty(len(C), dtype=np.int32)
    _load().orc_project(len(C), C.ctypes.data, cp.ctypes.data, out.ctypes.data)
    return out


def cut(g, part, k):
    """Returns (cut, block_weights int64[k])."""
    gv = _GraphView(g)
    p = np.ascontiguousarray(part, dtype=np.int32)
    c = np.zeros(1, dtype=np.int64)
    bw = np.zeros(k, dtype=np.int64)
    st = _load().orc_cut(gv.ref, p.ctypes.data, k, c.ctypes.data, bw.ctypes.data)
    if st != 0:
        raise ValueError("orc_cut status %d" % st)
    return int(c[0]), bw


def initial_partition(g, k, T):
    gv = _GraphView(g)
    part = np.empty(gv.n, dtype=np.int32)
    _load().orc_initial_partition(gv.ref, k, T, part.ctypes.data)
    return part


def initial_partition_lp(g, k, T, Lmax, seed=1, level=0, rounds=10, nsub=4):
    """Initial partition by label propagation from hashed seeds with a pool
    label.  Returns (part, rounds_run, visits)."""
    gv = _GraphView(g)
    part = np.empty(gv.n, dtype=np.int32)
    rr = np.zeros(1, dtype=np.int32)
    visits = np.zeros(1, dtype=np.int64)
    st = _load().orc_initial_partition_lp(gv.ref, k, T, Lmax, seed, level, rounds, nsub, part.ctypes.data,
                                          rr.ctypes.data, visits.ctypes.data)
    if st != 0:
        raise ValueError("orc_initial_partition_lp status %d" % st)
    return part, int(rr[0]), int(visits[0])


def default_options(**kw):
    o = Options()
    _load().orc_default_options(ctypes.byref(o))
    for key, val in kw.items():
        setattr(o, key, int(val))
    return o


def partition(g, k, eps=0.03, seed=1, **opts):
    """Full multilevel partition.  Returns dict with part, cut, block_weights,
    status, levels, visits, level_n, level_S, cluster_rounds, refine_rounds."""
    gv = _GraphView(g)
    o = default_options(**opts)
    part = np.empty(gv.n, dtype=np.int32)
    c = np.zeros(1, dtype=np.int64)
    bw = np.zeros(k, dtype=np.int64)
    st = _Stats()
    status = _load().orc_partition(gv.ref, k, eps, seed, ctypes.byref(o), part.ctypes.data, c.ctypes.data,
                                   bw.ctypes.data, ctypes.byref(st))
    if status < 0:
        raise ValueError("orc_partition status %d" % status)
    L = st.levels
    return {"part": part, "cut": int(c[0]), "block_weights": bw, "status": int(status), "levels": L,
            "visits": int(st.visits), "level_n": list(st.level_n[:L + 1]), "level_S": list(st.level_S[:L + 1]),
            "cluster_rounds": list(st.cluster_rounds[:L]), "refine_rounds": list(st.refine_rounds[:L + 1])}
