"""Python binding of libsclap.so (include/sclap.h): argument marshalling only.

Every step of the computation runs in the gfx950 kernels of the library; this
module only passes pointers and sizes through ctypes.  Host variants take
numpy arrays; ``*_dev`` variants take torch tensors on the GPU and enqueue on
the current torch stream (or the stream passed in).  A missing library raises
``ImportError``/``OSError``: there is no fallback path.

Graphs are dicts ``{"n", "xadj" int64[n+1], "adjncy" int32[S], "adjwgt"
int32[S] or None, "vwgt" int32[n] or None}`` of numpy arrays (host) or torch
tensors (device, see :func:`to_device`).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsclap.so")
_lib = None

OK, WARN_IMBALANCED = 0, 1
ERR_INVALID, ERR_NOT_SYMMETRIC, ERR_OVERFLOW, ERR_NO_MEMORY, ERR_HIP, ERR_BUSY = -1, -2, -3, -4, -5, -6
MAX_LEVELS = 64

#: every entry point declared in include/sclap.h
EXPORTS = [
    "sclap_default_options", "sclap_last_error", "sclap_lmax",
    "sclap_validate", "sclap_validate_dev",
    "sclap_cluster", "sclap_cluster_dev", "sclap_cluster_within", "sclap_cluster_within_dev",
    "sclap_contract", "sclap_contract_dev", "sclap_graph_free",
    "sclap_project", "sclap_project_dev",
    "sclap_refine", "sclap_refine_dev",
    "sclap_cut", "sclap_cut_dev", "sclap_cut_dev_noalloc",
    "sclap_initial_partition",
    "sclap_partition", "sclap_partition_dev",
    "sclap_partition_batch", "sclap_partition_batch_dev",
    "sclap_server_create", "sclap_server_submit", "sclap_server_poll", "sclap_server_destroy",
    "sclap_server_plan_batch",
    "sclap_autotune_dev", "sclap_trim_memory", "sclap_initial_partition_lp_dev",
    "sclap_profile_begin", "sclap_profile_end", "sclap_profile_begin_only", "sclap_gather_probe_dev",
]


class SclapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("sclap status %d: %s" % (status, msg))
        self.status = status


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xadj", ctypes.c_void_p), ("adjncy", ctypes.c_void_p),
                ("vwgt", ctypes.c_void_p), ("adjwgt", ctypes.c_void_p)]


class GraphOwned(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("S", ctypes.c_int64), ("xadj", ctypes.c_void_p),
                ("adjncy", ctypes.c_void_p), ("vwgt", ctypes.c_void_p), ("adjwgt", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("coarsen_rounds", ctypes.c_int32), ("refine_rounds", ctypes.c_int32),
                ("subrounds", ctypes.c_int32), ("cluster_divisor", ctypes.c_int32),
                ("coarsest_nodes", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("color_override", ctypes.c_void_p),
                ("lane_max_degree", ctypes.c_int32), ("wave_max_degree", ctypes.c_int32),
                ("block_max_degree", ctypes.c_int32), ("hub_part_limit", ctypes.c_int32),
                ("hub_region_cap", ctypes.c_int32), ("select_small_max", ctypes.c_int32),
                ("skip_quiet", ctypes.c_int32), ("vcycles", ctypes.c_int32),
                ("degree_order", ctypes.c_int32), ("contract_bucket_mean", ctypes.c_int32),
                ("initial_partitioner", ctypes.c_int32), ("select_launches", ctypes.c_int32),
                ("graph_capture", ctypes.c_int32), ("fused_eval", ctypes.c_int32),
                ("block_table", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("visits", ctypes.c_int64),
                ("level_n", ctypes.c_int32 * (MAX_LEVELS + 1)), ("level_S", ctypes.c_int64 * (MAX_LEVELS + 1)),
                ("cluster_rounds", ctypes.c_int32 * (MAX_LEVELS + 1)),
                ("refine_rounds", ctypes.c_int32 * (MAX_LEVELS + 1)),
                ("ms_coarsen", ctypes.c_double), ("ms_initial", ctypes.c_double),
                ("ms_refine", ctypes.c_double), ("ms_lp", ctypes.c_double)]

    def to_dict(self):
        L = self.levels
        return {"levels": L, "visits": self.visits, "level_n": list(self.level_n[:L + 1]),
                "level_S": list(self.level_S[:L + 1]), "cluster_rounds": list(self.cluster_rounds[:L]),
                "refine_rounds": list(self.refine_rounds[:L + 1]), "ms_coarsen": self.ms_coarsen,
                "ms_initial": self.ms_initial, "ms_refine": self.ms_refine, "ms_lp": self.ms_lp}


class BatchStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("visits", ctypes.c_int64),
                ("ms_coarsen", ctypes.c_double), ("ms_initial", ctypes.c_double),
                ("ms_refine", ctypes.c_double), ("ms_lp", ctypes.c_double),
                ("graph_levels", ctypes.c_void_p)]

    def to_dict(self):
        return {"levels": self.levels, "visits": self.visits, "ms_coarsen": self.ms_coarsen,
                "ms_initial": self.ms_initial, "ms_refine": self.ms_refine, "ms_lp": self.ms_lp}


class RequestInfo(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("batch_size", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def load():
    """Loads libsclap.so (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsclap.so not built: run __graft_entry__.build() (%s)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    G = ctypes.POINTER(Graph)
    O = ctypes.POINTER(Options)
    GO = ctypes.POINTER(GraphOwned)
    ST = ctypes.POINTER(Stats)
    BST = ctypes.POINTER(BatchStats)
    sig = {
        "sclap_default_options": (ctypes.c_int, [O]),
        "sclap_last_error": (ctypes.c_char_p, []),
        "sclap_lmax": (i64, [i64, i32, dbl]),
        "sclap_validate": (ctypes.c_int, [G]),
        "sclap_validate_dev": (ctypes.c_int, [G, vp]),
        "sclap_cluster": (ctypes.c_int, [G, i64, i32, u64, i32, O, vp, vp]),
        "sclap_cluster_dev": (ctypes.c_int, [G, i64, i32, u64, i32, O, vp, vp, vp]),
        "sclap_cluster_within": (ctypes.c_int, [G, vp, i64, i32, u64, i32, O, vp, vp]),
        "sclap_cluster_within_dev": (ctypes.c_int, [G, vp, i64, i32, u64, i32, O, vp, vp, vp]),
        "sclap_contract": (ctypes.c_int, [G, vp, vp, GO]),
        "sclap_contract_dev": (ctypes.c_int, [G, vp, vp, GO, vp]),
        "sclap_graph_free": (None, [GO]),
        "sclap_project": (ctypes.c_int, [i32, i32, vp, vp, vp]),
        "sclap_project_dev": (ctypes.c_int, [i32, i32, vp, vp, vp, vp]),
        "sclap_refine": (ctypes.c_int, [G, i32, i64, i32, u64, i32, O, vp, vp]),
        "sclap_refine_dev": (ctypes.c_int, [G, i32, i64, i32, u64, i32, O, vp, vp, vp]),
        "sclap_cut": (ctypes.c_int, [G, vp, i32, vp, vp]),
        "sclap_cut_dev": (ctypes.c_int, [G, vp, i32, vp, vp, vp]),
        "sclap_cut_dev_noalloc": (ctypes.c_int, [G, vp, i32, vp, vp, vp]),
        "sclap_initial_partition": (ctypes.c_int, [G, i32, vp]),
        "sclap_partition": (ctypes.c_int, [G, i32, dbl, u64, O, vp, vp, vp, ST]),
        "sclap_partition_dev": (ctypes.c_int, [G, i32, dbl, u64, O, vp, vp, vp, ST, vp]),
        "sclap_partition_batch": (ctypes.c_int, [G, i32, vp, vp, vp, vp, O, vp, vp, vp, BST]),
        "sclap_server_create": (vp, [i32, i64, i32, i32, O]),
        "sclap_server_submit": (ctypes.c_int, [vp, G, i32, dbl, u64, vp]),
        "sclap_server_poll": (ctypes.c_int, [vp, u64, i32, vp, vp, vp, vp, ctypes.POINTER(RequestInfo)]),
        "sclap_server_destroy": (None, [vp]),
        "sclap_autotune_dev": (ctypes.c_int, [G, i32, O, vp]),
        "sclap_trim_memory": (ctypes.c_int, []),
        "sclap_initial_partition_lp_dev": (ctypes.c_int, [G, i32, i64, i64, u64, i32, i32, O, vp, vp, vp]),
        "sclap_partition_batch_dev": (ctypes.c_int, [G, i32, vp, vp, vp, vp, O, vp, vp, vp, BST, vp]),
        "sclap_profile_begin": (ctypes.c_int, []),
        "sclap_profile_begin_only": (ctypes.c_int, [ctypes.c_char_p]),
        "sclap_profile_end": (ctypes.c_int, [ctypes.POINTER(KernelStat), i32, vp]),
        "sclap_gather_probe_dev": (ctypes.c_int, [G, i32, i32, vp, vp]),
        "sclap_server_plan_batch": (ctypes.c_int32, [vp, vp, vp, i32, i64, i32, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error():
    return load().sclap_last_error().decode()


def _check(st, allow_warn=False):
    if st < 0 or (st > 0 and not allow_warn):
        raise SclapError(st, last_error())
    return st


def default_options(**kw):
    o = Options()
    load().sclap_default_options(ctypes.byref(o))
    for key, val in kw.items():
        setattr(o, key, val)
    return o


def lmax(cV, k, eps):
    return int(load().sclap_lmax(cV, k, eps))


# ----------------------------------------------------------------- host side

def _np_ptr(a):
    return None if a is None else a.ctypes.data


class _HostGraph:
    def __init__(self, g):
        self.xadj = np.ascontiguousarray(g["xadj"], dtype=np.int64)
        self.adjncy = np.ascontiguousarray(g["adjncy"], dtype=np.int32)
        self.vwgt = None if g.get("vwgt") is None else np.ascontiguousarray(g["vwgt"], dtype=np.int32)
        self.adjwgt = None if g.get("adjwgt") is None else np.ascontiguousarray(g["adjwgt"], dtype=np.int32)
        self.n = int(g["n"])
        self.s = Graph(self.n, _np_ptr(self.xadj), _np_ptr(self.adjncy), _np_ptr(self.vwgt), _np_ptr(self.adjwgt))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _opts(opts, color_override=None, keep=None):
    o = opts if isinstance(opts, Options) else default_options(**(opts or {}))
    if color_override is not None:
        o.color_override = color_override
    return o


def validate(g):
    return int(load().sclap_validate(_HostGraph(g).ref))


def cluster(g, U, rounds=10, seed=1, level=0, color_override=None, block=None, **opts):
    """Size-constrained clustering; with ``block`` (int32[n]) only inside the
    blocks of that partition.  Returns (labels, rounds_run)."""
    hg = _HostGraph(g)
    co = None if color_override is None else np.ascontiguousarray(color_override, dtype=np.int32)
    o = _opts(opts, _np_ptr(co))
    labels = np.empty(hg.n, dtype=np.int32)
    rr = ctypes.c_int32(0)
    if block is None:
        _check(load().sclap_cluster(hg.ref, U, rounds, seed, level, ctypes.byref(o), labels.ctypes.data,
                                    ctypes.addressof(rr)))
    else:
        blk = np.ascontiguousarray(block, dtype=np.int32)
        _check(load().sclap_cluster_within(hg.ref, blk.ctypes.data, U, rounds, seed, level, ctypes.byref(o),
                                           labels.ctypes.data, ctypes.addressof(rr)))
    return labels, rr.value


def refine(g, k, Lmax, part, rounds=10, seed=1, level=0, color_override=None, **opts):
    hg = _HostGraph(g)
    co = None if color_override is None else np.ascontiguousarray(color_override, dtype=np.int32)
    o = _opts(opts, _np_ptr(co))
    p = np.array(part, dtype=np.int32, copy=True)
    rr = ctypes.c_int32(0)
    _check(load().sclap_refine(hg.ref, k, Lmax, rounds, seed, level, ctypes.byref(o), p.ctypes.data,
                               ctypes.addressof(rr)))
    return p, rr.value


def contract(g, labels):
    hg = _HostGraph(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    C = np.empty(hg.n, dtype=np.int32)
    out = GraphOwned()
    L = load()
    _check(L.sclap_contract(hg.ref, lab.ctypes.data, C.ctypes.data, ctypes.byref(out)))
    try:
        n, S = out.n, out.S
        def arr(ptr, count, ct, dt):
            if count == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(count,)).copy()
        cg = {"n": n, "xadj": arr(out.xadj, n + 1, ctypes.c_int64, np.int64),
              "adjncy": arr(out.adjncy, S, ctypes.c_int32, np.int32),
              "adjwgt": arr(out.adjwgt, S, ctypes.c_int32, np.int32),
              "vwgt": arr(out.vwgt, n, ctypes.c_int32, np.int32)}
    finally:
        L.sclap_graph_free(ctypes.byref(out))
    return C, cg


def project(C, coarse_part):
    C = np.ascontiguousarray(C, dtype=np.int32)
    cp = np.ascontiguousarray(coarse_part, dtype=np.int32)
    out = np.empty(len(C), dtype=np.int32)
    _check(load().sclap_project(len(C), len(cp), C.ctypes.data, cp.ctypes.data, out.ctypes.data))
    return out


def cut(g, part, k):
    hg = _HostGraph(g)
    p = np.ascontiguousarray(part, dtype=np.int32)
    c = ctypes.c_int64(0)
    bw = np.zeros(k, dtype=np.int64)
    _check(load().sclap_cut(hg.ref, p.ctypes.data, k, ctypes.addressof(c), bw.ctypes.data))
    return c.value, bw


def initial_partition(g, k):
    hg = _HostGraph(g)
    part = np.empty(hg.n, dtype=np.int32)
    _check(load().sclap_initial_partition(hg.ref, k, part.ctypes.data))
    return part


def partition(g, k, eps=0.03, seed=1, **opts):
    """Multilevel partition of a host graph; returns dict(part, cut,
    block_weights, status, stats)."""
    hg = _HostGraph(g)
    o = _opts(opts)
    part = np.empty(hg.n, dtype=np.int32)
    c = ctypes.c_int64(0)
    bw = np.zeros(k, dtype=np.int64)
    st = Stats()
    status = _check(load().sclap_partition(hg.ref, k, eps, seed, ctypes.byref(o), part.ctypes.data,
                                           ctypes.addressof(c), bw.ctypes.data, ctypes.byref(st)),
                    allow_warn=True)
    return {"part": part, "cut": c.value, "block_weights": bw, "status": status, "stats": st.to_dict()}


# --------------------------------------------------------------- device side

def to_device(g, device="cuda"):
    """Copies a host graph dict to torch tensors on the GPU."""
    import torch
    d = {"n": int(g["n"]), "xadj": torch.as_tensor(np.ascontiguousarray(g["xadj"], dtype=np.int64)).to(device),
         "adjncy": torch.as_tensor(np.ascontiguousarray(g["adjncy"], dtype=np.int32)).to(device)}
    for key in ("adjwgt", "vwgt"):
        d[key] = None if g.get(key) is None else torch.as_tensor(
            np.ascontiguousarray(g[key], dtype=np.int32)).to(device)
    return d


def _t_ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class _DevGraph:
    def __init__(self, d):
        for key in ("xadj", "adjncy", "adjwgt", "vwgt"):
            t = d.get(key)
            if t is not None:
                assert t.is_cuda and t.is_contiguous(), key
        assert d["xadj"].dtype.itemsize == 8 and d["adjncy"].dtype.itemsize == 4
        self.d = d
        self.n = int(d["n"])
        self.s = Graph(self.n, _t_ptr(d["xadj"]), _t_ptr(d["adjncy"]), _t_ptr(d.get("vwgt")),
                       _t_ptr(d.get("adjwgt")))

    @property
    def ref(self):
        return ctypes.byref(self.s)


def validate_dev(d, stream=None):
    return int(load().sclap_validate_dev(_DevGraph(d).ref, _stream(stream)))


def cluster_dev(d, U, rounds=10, seed=1, level=0, labels=None, color_override=None, stream=None, block=None,
                **opts):
    """cluster() on a device graph; ``block`` is an int32 tensor on the GPU."""
    import torch
    dg = _DevGraph(d)
    if labels is None:
        labels = torch.empty(dg.n, dtype=torch.int32, device=d["xadj"].device)
    o = _opts(opts, _t_ptr(color_override))
    rr = ctypes.c_int32(0)
    if block is None:
        _check(load().sclap_cluster_dev(dg.ref, U, rounds, seed, level, ctypes.byref(o), _t_ptr(labels),
                                        ctypes.addressof(rr), _stream(stream)))
    else:
        _check(load().sclap_cluster_within_dev(dg.ref, _t_ptr(block), U, rounds, seed, level, ctypes.byref(o),
                                               _t_ptr(labels), ctypes.addressof(rr), _stream(stream)))
    return labels, rr.value


def refine_dev(d, k, Lmax, part, rounds=10, seed=1, level=0, color_override=None, stream=None, **opts):
    """Refines ``part`` (int32 tensor on the GPU) in place."""
    dg = _DevGraph(d)
    o = _opts(opts, _t_ptr(color_override))
    rr = ctypes.c_int32(0)
    _check(load().sclap_refine_dev(dg.ref, k, Lmax, rounds, seed, level, ctypes.byref(o), _t_ptr(part),
                                   ctypes.addressof(rr), _stream(stream)))
    return part, rr.value


def contract_dev(d, labels, stream=None):
    """Returns (C tensor, coarse graph dict of tensors copied from the library's buffers)."""
    import torch
    dg = _DevGraph(d)
    dev = d["xadj"].device
    C = torch.empty(dg.n, dtype=torch.int32, device=dev)
    out = GraphOwned()
    L = load()
    _check(L.sclap_contract_dev(dg.ref, _t_ptr(labels), _t_ptr(C), ctypes.byref(out), _stream(stream)))
    try:
        n, S = out.n, out.S
        cg = {"n": n, "xadj": torch.empty(n + 1, dtype=torch.int64, device=dev),
              "adjncy": torch.empty(S, dtype=torch.int32, device=dev),
              "adjwgt": torch.empty(S, dtype=torch.int32, device=dev),
              "vwgt": torch.empty(n, dtype=torch.int32, device=dev)}
        import torch.cuda as tc
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        tc.synchronize()
        for key, ptr, nb in (("xadj", out.xadj, (n + 1) * 8), ("adjncy", out.adjncy, S * 4),
                             ("adjwgt", out.adjwgt, S * 4), ("vwgt", out.vwgt, n * 4)):
            if nb > 0 and ptr:
                rc = hip.hipMemcpy(cg[key].data_ptr(), ptr, nb, 3)  # device to device
                if rc != 0:
                    raise SclapError(ERR_HIP, "hipMemcpy failed (%d)" % rc)
    finally:
        L.sclap_graph_free(ctypes.byref(out))
    return C, cg


def project_dev(C, coarse_part, part=None, stream=None):
    import torch
    if part is None:
        part = torch.empty_like(C)
    _check(load().sclap_project_dev(C.numel(), coarse_part.numel(), _t_ptr(C), _t_ptr(coarse_part), _t_ptr(part),
                                    _stream(stream)))
    return part


def cut_dev(d, part, k, stream=None):
    dg = _DevGraph(d)
    c = ctypes.c_int64(0)
    bw = np.zeros(k, dtype=np.int64)
    _check(load().sclap_cut_dev(dg.ref, _t_ptr(part), k, ctypes.addressof(c), bw.ctypes.data, _stream(stream)))
    return c.value, bw


def cut_dev_noalloc(d, part, k, stream=None):
    """As cut_dev, through the entry point that allocates no device memory."""
    dg = _DevGraph(d)
    c = ctypes.c_int64(0)
    bw = np.zeros(k, dtype=np.int64)
    _check(load().sclap_cut_dev_noalloc(dg.ref, _t_ptr(part), k, ctypes.addressof(c), bw.ctypes.data,
                                        _stream(stream)))
    return c.value, bw


def partition_dev(d, k, eps=0.03, seed=1, part=None, stream=None, opts=None, **kw):
    """Multilevel partition of a device graph; ``part`` (int32 tensor) receives
    the blocks.  Returns dict(part, cut, block_weights, status, stats)."""
    import torch
    dg = _DevGraph(d)
    if part is None:
        part = torch.empty(dg.n, dtype=torch.int32, device=d["xadj"].device)
    o = opts if isinstance(opts, Options) else default_options(**kw)
    c = ctypes.c_int64(0)
    bw = np.zeros(k, dtype=np.int64)
    st = Stats()
    status = _check(load().sclap_partition_dev(dg.ref, k, eps, seed, ctypes.byref(o), _t_ptr(part),
                                               ctypes.addressof(c), bw.ctypes.data, ctypes.byref(st),
                                               _stream(stream)), allow_warn=True)
    return {"part": part, "cut": c.value, "block_weights": bw, "status": status, "stats": st.to_dict()}


def profile_begin(only=None):
    """Starts per-kernel HIP-event timing of the library's launches on this
    thread; with ``only``, of that kernel's launches alone."""
    if only:
        _check(load().sclap_profile_begin_only(only.encode()))
    else:
        _check(load().sclap_profile_begin())


def profile_end():
    """Stops timing; returns {kernel name: dict(launches, ms, bytes)}."""
    cap = 64
    arr = (KernelStat * cap)()
    cnt = ctypes.c_int32(0)
    _check(load().sclap_profile_end(arr, cap, ctypes.addressof(cnt)))
    return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].ms, "bytes": arr[i].bytes}
            for i in range(min(cnt.value, cap))}


def gather_probe_dev(d, label_bytes=4, reps=3, stream=None):
    """Average ms of one pass gathering label[adj[e]] over every slot of the
    device graph ``d`` (1- or 4-byte labels)."""
    dg = _DevGraph(d)
    ms = ctypes.c_double(0)
    _check(load().sclap_gather_probe_dev(dg.ref, label_bytes, reps, ctypes.addressof(ms), _stream(stream)))
    return ms.value


# ------------------------------------------------------------------ batches

def union(graphs):
    """Concatenates host graph dicts into one CSR (graph i's ids shifted by
    the nodes before it).  Returns (graph dict, node_base int32[count+1])."""
    nb = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        nb[i + 1] = nb[i] + int(g["n"])
    if nb[-1] > np.iinfo(np.int32).max:
        raise ValueError("batch has more than 2^31-1 nodes")
    S = [int(g["xadj"][-1]) if int(g["n"]) > 0 else 0 for g in graphs]
    sb = np.concatenate([[0], np.cumsum(S)]).astype(np.int64)
    xadj = np.zeros(int(nb[-1]) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        if int(g["n"]) > 0:
            xadj[nb[i] + 1:nb[i + 1] + 1] = np.asarray(g["xadj"][1:], dtype=np.int64) + sb[i]
    adj = np.concatenate([np.asarray(g["adjncy"][:S[i]], dtype=np.int64) + nb[i] for i, g in enumerate(graphs)]
                         or [np.zeros(0, dtype=np.int64)]).astype(np.int32)
    u = {"n": int(nb[-1]), "xadj": xadj, "adjncy": adj}
    for key, size in (("adjwgt", S), ("vwgt", [int(g["n"]) for g in graphs])):
        if all(g.get(key) is None for g in graphs):
            u[key] = None
        else:
            u[key] = np.concatenate([np.ones(size[i], dtype=np.int32) if g.get(key) is None
                                     else np.asarray(g[key][:size[i]], dtype=np.int32)
                                     for i, g in enumerate(graphs)] or [np.zeros(0, dtype=np.int32)])
    return u, nb.astype(np.int32)


def _batch_args(count, k, eps, seed):
    k = np.ascontiguousarray(k, dtype=np.int32)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    seed = np.ascontiguousarray(seed, dtype=np.uint64)
    if not (len(k) == len(eps) == len(seed) == count):
        raise ValueError("k, eps and seed need one entry per graph")
    return k, eps, seed


def _split_batch(part, node_base, k, cut, bw, status, st, levels):
    kb = np.concatenate([[0], np.cumsum(k)])
    out = []
    for i in range(len(k)):
        out.append({"part": part[node_base[i]:node_base[i + 1]], "cut": int(cut[i]),
                    "block_weights": bw[kb[i]:kb[i + 1]], "levels": int(levels[i])})
    return {"graphs": out, "status": status, "stats": st.to_dict()}


def partition_batch(graphs, k, eps, seed, **opts):
    """Partitions a list of host graphs together (one multilevel pass over
    their union).  Returns dict(graphs=[dict(part, cut, block_weights,
    levels)], status, stats); each graph's result equals partition() of that
    graph alone."""
    g, node_base = union(graphs)
    return partition_batch_union(g, node_base, k, eps, seed, **opts)


def partition_batch_union(g, node_base, k, eps, seed, **opts):
    """partition_batch() on a host union already built (see union())."""
    node_base = np.ascontiguousarray(node_base, dtype=np.int32)
    count = len(node_base) - 1
    k, eps, seed = _batch_args(count, k, eps, seed)
    hg = _HostGraph(g)
    o = _opts(opts)
    part = np.empty(hg.n, dtype=np.int32)
    cut = np.zeros(count, dtype=np.int64)
    bw = np.zeros(int(k.sum()), dtype=np.int64)
    levels = np.zeros(count, dtype=np.int32)
    st = BatchStats()
    st.graph_levels = levels.ctypes.data
    status = _check(load().sclap_partition_batch(hg.ref, count, node_base.ctypes.data, k.ctypes.data,
                                                 eps.ctypes.data, seed.ctypes.data, ctypes.byref(o),
                                                 part.ctypes.data, cut.ctypes.data, bw.ctypes.data,
                                                 ctypes.byref(st)), allow_warn=True)
    return _split_batch(part, node_base, k, cut, bw, status, st, levels)


def partition_batch_dev(d, node_base, k, eps, seed, part=None, stream=None, opts=None, **kw):
    """Batched partition of a device-resident union (see union()); ``part``
    receives graph-local blocks.  Returns dict(part, cut[count],
    block_weights[sum k], levels[count], status, stats)."""
    import torch
    dg = _DevGraph(d)
    node_base = np.ascontiguousarray(node_base, dtype=np.int32)
    count = len(node_base) - 1
    k, eps, seed = _batch_args(count, k, eps, seed)
    if part is None:
        part = torch.empty(dg.n, dtype=torch.int32, device=d["xadj"].device)
    o = opts if isinstance(opts, Options) else default_options(**kw)
    cut = np.zeros(count, dtype=np.int64)
    bw = np.zeros(int(k.sum()), dtype=np.int64)
    levels = np.zeros(count, dtype=np.int32)
    st = BatchStats()
    st.graph_levels = levels.ctypes.data
    status = _check(load().sclap_partition_batch_dev(dg.ref, count, node_base.ctypes.data, k.ctypes.data,
                                                     eps.ctypes.data, seed.ctypes.data, ctypes.byref(o),
                                                     _t_ptr(part), cut.ctypes.data, bw.ctypes.data,
                                                     ctypes.byref(st), _stream(stream)), allow_warn=True)
    return {"part": part, "cut": cut, "block_weights": bw, "levels": levels, "status": status,
            "stats": st.to_dict()}


def initial_partition_lp_dev(d, k, T, Lmax, seed=1, level=0, rounds=10, part=None, stream=None, **opts):
    """Device initial partitioner on a device graph; returns (part tensor, visits)."""
    import torch
    dg = _DevGraph(d)
    if part is None:
        part = torch.empty(max(dg.n, 1), dtype=torch.int32, device=d["xadj"].device)
    o = _opts(opts)
    visits = ctypes.c_int64(0)
    _check(load().sclap_initial_partition_lp_dev(dg.ref, k, T, Lmax, seed, level, rounds, ctypes.byref(o),
                                                 _t_ptr(part), ctypes.addressof(visits), _stream(stream)))
    return part[:dg.n], visits.value


def autotune_dev(d, k, stream=None, opts=None, **kw):
    """Returns Options whose tuning fields (degree-bucket thresholds, the
    longest-row workgroup bucket's table size, graph capture) ran one
    clustering and one refinement round of the device graph ``d`` fastest
    (results never depend on them)."""
    dg = _DevGraph(d)
    o = opts if isinstance(opts, Options) else default_options(**kw)
    _check(load().sclap_autotune_dev(dg.ref, k, ctypes.byref(o), _stream(stream)))
    return o


# ------------------------------------------------------------------ serving

def server_plan_batch(nodes, slots, footprint, free_budget, max_batch, idle=True):
    """The server's batch-packing rule: how many of the queued requests
    (node counts, slot counts, footprints in queue order) one batch takes."""
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    slots = np.ascontiguousarray(slots, dtype=np.int64)
    footprint = np.ascontiguousarray(footprint, dtype=np.int64)
    r = load().sclap_server_plan_batch(nodes.ctypes.data, slots.ctypes.data, footprint.ctypes.data, len(nodes),
                                       free_budget, max_batch, int(bool(idle)))
    if r < 0:
        raise SclapError(r, "invalid arguments")
    return int(r)


class Server:
    """Continuous-batching partition server on one GPU (see sclap.h).

    submit() copies the graph and returns a request id; poll() returns None
    while the request runs, else dict(part, cut, block_weights, status,
    submit_ms, start_ms, done_ms, batch_size).  A failed request raises
    SclapError from poll()."""

    def __init__(self, device=0, hbm_budget=0, slots=2, max_batch=64, **opts):
        L = load()
        self._o = _opts(opts)
        self._p = L.sclap_server_create(device, hbm_budget, slots, max_batch, ctypes.byref(self._o))
        if not self._p:
            raise SclapError(ERR_INVALID, last_error())
        self._meta = {}

    def submit(self, g, k, eps=0.03, seed=1):
        hg = _HostGraph(g)
        rid = ctypes.c_uint64(0)
        _check(load().sclap_server_submit(self._p, hg.ref, k, eps, seed, ctypes.addressof(rid)))
        self._meta[rid.value] = (hg.n, k)
        return rid.value

    def poll(self, rid, timeout_ms=0):
        n, k = self._meta[rid]
        done = ctypes.c_int32(0)
        part = np.empty(max(n, 1), dtype=np.int32)
        cut = ctypes.c_int64(0)
        bw = np.zeros(k, dtype=np.int64)
        info = RequestInfo()
        try:
            status = _check(load().sclap_server_poll(self._p, rid, timeout_ms, ctypes.addressof(done),
                                                     part.ctypes.data, ctypes.addressof(cut), bw.ctypes.data,
                                                     ctypes.byref(info)), allow_warn=True)
        except SclapError:
            self._meta.pop(rid, None)
            raise
        if not done.value:
            return None
        del self._meta[rid]
        return {"part": part[:n], "cut": cut.value, "block_weights": bw, "status": status,
                "submit_ms": info.submit_ms, "start_ms": info.start_ms, "done_ms": info.done_ms,
                "batch_size": info.batch_size}

    def wait(self, rid):
        return self.poll(rid, timeout_ms=-1)

    def close(self):
        if self._p:
            load().sclap_server_destroy(self._p)
            self._p = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
