"""Python binding of libknngmerge.so (include/knng_merge.h).

Argument marshalling only: every step of every call runs in the HIP kernels of
the library.  PyTorch provides device memory (inputs, outputs, workspace) and
the stream.  There is no fallback: if the library is not built, load() raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknngmerge.so")

L2, COSINE, L1 = 0, 1, 2
METRICS = {"l2": L2, "cos": COSINE, "cosine": COSINE, "l1": L1}
FP32, BF16_RESCORE = 0, 1
PRECISIONS = {"fp32": FP32, "bf16": BF16_RESCORE, "bf16_rescore": BF16_RESCORE}
FLAG_PROFILE = 1
FLAG_BALANCED_APPEND = 2
STATS_ROUNDS = 64

STATUS = {0: "KNNG_OK", 1: "KNNG_EINVAL", 2: "KNNG_ENOMEM", 3: "KNNG_EDEVICE", 4: "KNNG_EBUSY"}

ENTRY_POINTS = ["knng_opts_default", "knng_merge", "knng_merge_workspace_size", "knng_expand",
                "knng_expand_workspace_size", "knng_merge_bruteforce",
                "knng_bruteforce_workspace_size", "knng_exact_graph",
                "knng_exact_graph_workspace_size", "knng_last_error", "knng_version",
                "knng_merge_tree", "knng_merge_tree_workspace_size", "knng_hmerge",
                "knng_hmerge_workspace_size", "knng_server_bytes",
                "knng_server_create", "knng_server_submit", "knng_server_step",
                "knng_server_wait", "knng_server_snapshot", "knng_server_rebase",
                "knng_server_status", "knng_server_slots", "knng_server_destroy",
                "knng_merge_noalloc", "knng_merge_noalloc_scratch_bytes",
                "knng_hierarchy_shape", "knng_hmerge_hierarchy", "knng_diversify",
                "knng_diversify_workspace_size", "knng_search", "knng_search_workspace_size",
                "knng_server_fail_request"]


class Opts(ctypes.Structure):
    _fields_ = [("keep_ratio", ctypes.c_float), ("sample", ctypes.c_int32),
                ("delta", ctypes.c_float), ("max_rounds", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class Set(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("x", ctypes.c_void_p)]


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int32), ("ids", ctypes.c_void_p),
                ("dist", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("max_group", ctypes.c_int32),
                ("evals", ctypes.c_int64), ("rescored", ctypes.c_int64),
                ("insert_attempts", ctypes.c_int64), ("screen_violations", ctypes.c_int64),
                ("updates", ctypes.c_int64 * STATS_ROUNDS),
                ("pairs", ctypes.c_int64 * STATS_ROUNDS),
                ("gathered", ctypes.c_int64 * STATS_ROUNDS),
                ("ms_prep", ctypes.c_double), ("ms_init", ctypes.c_double),
                ("ms_sample", ctypes.c_double), ("ms_reverse", ctypes.c_double),
                ("ms_join", ctypes.c_double), ("ms_final", ctypes.c_double),
                ("join_launches", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def to_dict(self):
        r = min(self.rounds, STATS_ROUNDS)
        return {"rounds": self.rounds, "max_group": self.max_group, "evals": self.evals,
                "rescored": self.rescored, "insert_attempts": self.insert_attempts,
                "screen_violations": self.screen_violations,
                "c": list(self.updates[:r]),
                "pairs": list(self.pairs[:r]), "gathered": list(self.gathered[:r]),
                "ms": {"prep": self.ms_prep, "init": self.ms_init, "sample": self.ms_sample,
                       "reverse": self.ms_reverse, "join": self.ms_join,
                       "final": self.ms_final},
                "join_launches": self.join_launches}


class ServerConfig(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("max_request", ctypes.c_int64),
                ("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_int32),
                ("batching", ctypes.c_int32), ("host_rounds", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("first_id", ctypes.c_int64), ("rows", ctypes.c_int64),
                ("merged_first", ctypes.c_int64), ("merged_rows", ctypes.c_int64),
                ("evals", ctypes.c_int64), ("rounds", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("submit_us", ctypes.c_double), ("start_us", ctypes.c_double),
                ("done_us", ctypes.c_double)]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KnngError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load the built library (raises if it is missing: no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1908_00814_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    pS, pG, pO, pSt = (ctypes.POINTER(Set), ctypes.POINTER(Graph), ctypes.POINTER(Opts),
                       ctypes.POINTER(Stats))
    lib.knng_opts_default.restype = None
    lib.knng_opts_default.argtypes = [pO]
    lib.knng_merge.restype = ctypes.c_int
    lib.knng_merge.argtypes = [pS, pG, pS, pG, I32, ctypes.c_int, pO, pG, P, SZ, P, pSt]
    lib.knng_hierarchy_shape.restype = I32
    lib.knng_hierarchy_shape.argtypes = [I64, I64, I32, P, P, I32]
    lib.knng_hmerge_hierarchy.restype = ctypes.c_int
    lib.knng_hmerge_hierarchy.argtypes = [pS, I32, I64, ctypes.c_int, pO, P, P, pG, I32, P, SZ,
                                          P, pSt]
    lib.knng_diversify.restype = ctypes.c_int
    lib.knng_diversify.argtypes = [pS, pG, I32, ctypes.c_int, pG, P, SZ, P]
    lib.knng_diversify_workspace_size.restype = SZ
    lib.knng_diversify_workspace_size.argtypes = [I64, I32, I32, ctypes.c_int]
    lib.knng_search.restype = ctypes.c_int
    lib.knng_search.argtypes = [pS, pG, I32, pS, I32, I32, ctypes.c_uint64, ctypes.c_int, P, P,
                                P, SZ, P, ctypes.POINTER(I64)]
    lib.knng_search_workspace_size.restype = SZ
    lib.knng_search_workspace_size.argtypes = [I64, I32, I64, ctypes.c_int]
    lib.knng_merge_noalloc.restype = ctypes.c_int
    lib.knng_merge_noalloc.argtypes = [pS, pG, pS, pG, I32, ctypes.c_int, pO, pG, P, pSt]
    lib.knng_merge_noalloc_scratch_bytes.restype = SZ
    lib.knng_merge_noalloc_scratch_bytes.argtypes = []
    lib.knng_merge_workspace_size.restype = SZ
    lib.knng_merge_workspace_size.argtypes = [I64, I64, I32, I32, I32, I32, ctypes.c_int, pO]
    lib.knng_expand.restype = ctypes.c_int
    lib.knng_expand.argtypes = [pS, pG, pS, I32, ctypes.c_int, pO, pG, P, SZ, P, pSt]
    lib.knng_expand_workspace_size.restype = SZ
    lib.knng_expand_workspace_size.argtypes = [I64, I64, I32, I32, I32, ctypes.c_int, pO]
    lib.knng_merge_bruteforce.restype = ctypes.c_int
    lib.knng_merge_bruteforce.argtypes = [pS, pG, pS, pG, I32, ctypes.c_int, pG, P, SZ, P]
    lib.knng_bruteforce_workspace_size.restype = SZ
    lib.knng_bruteforce_workspace_size.argtypes = [I64, I64, I32, I32, I32, I32, ctypes.c_int]
    lib.knng_exact_graph.restype = ctypes.c_int
    lib.knng_exact_graph.argtypes = [pS, I32, ctypes.c_int, pG, P, SZ, P]
    lib.knng_exact_graph_workspace_size.restype = SZ
    lib.knng_exact_graph_workspace_size.argtypes = [I64, I32, I32, ctypes.c_int]
    lib.knng_merge_tree.restype = ctypes.c_int
    lib.knng_merge_tree.argtypes = [pS, P, pG, I32, I32, ctypes.c_int, pO, pG, P, SZ, P, pSt]
    lib.knng_merge_tree_workspace_size.restype = SZ
    lib.knng_merge_tree_workspace_size.argtypes = [I64, I32, I32, P, I32, I32, ctypes.c_int, pO]
    lib.knng_hmerge.restype = ctypes.c_int
    lib.knng_hmerge.argtypes = [pS, I32, I64, ctypes.c_int, pO, pG, P, SZ, P, pSt]
    lib.knng_hmerge_workspace_size.restype = SZ
    lib.knng_hmerge_workspace_size.argtypes = [I64, I32, I32, I64, ctypes.c_int, pO]
    lib.knng_server_bytes.restype = SZ
    lib.knng_server_bytes.argtypes = [I64, I64, I32, I32, I32, ctypes.c_int, pO, I32]
    lib.knng_server_create.restype = ctypes.c_int
    lib.knng_server_create.argtypes = [pS, pG, I32, ctypes.c_int, pO,
                                       ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
    lib.knng_server_submit.restype = ctypes.c_int
    lib.knng_server_submit.argtypes = [P, P, I64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.knng_server_step.restype = ctypes.c_int
    lib.knng_server_step.argtypes = [P, ctypes.POINTER(I32)]
    lib.knng_server_wait.restype = ctypes.c_int
    lib.knng_server_wait.argtypes = [P, ctypes.c_uint64, I64, P, P, ctypes.POINTER(RequestInfo)]
    lib.knng_server_snapshot.restype = ctypes.c_int
    lib.knng_server_snapshot.argtypes = [P, pG, ctypes.POINTER(I64)]
    lib.knng_server_rebase.restype = ctypes.c_int
    lib.knng_server_rebase.argtypes = [P]
    lib.knng_server_slots.restype = I32
    lib.knng_server_slots.argtypes = [P]
    lib.knng_server_status.restype = ctypes.c_int
    lib.knng_server_status.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                       ctypes.POINTER(I64)]
    lib.knng_server_fail_request.restype = ctypes.c_int
    lib.knng_server_fail_request.argtypes = [P, ctypes.c_uint64]
    lib.knng_server_destroy.restype = None
    lib.knng_server_destroy.argtypes = [P]
    lib.knng_last_error.restype = ctypes.c_char_p
    lib.knng_last_error.argtypes = []
    lib.knng_version.restype = ctypes.c_int
    lib.knng_version.argtypes = []
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise KnngError(rc, load().knng_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _set(x):
    assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 2
    return Set(x.shape[0], x.shape[1], x.data_ptr())


def _graph(ids, dist):
    assert ids.is_cuda and ids.dtype == torch.int32 and ids.is_contiguous()
    if dist is not None:
        assert dist.is_cuda and dist.dtype == torch.float32 and dist.is_contiguous()
    return Graph(ids.shape[0], ids.shape[1], ids.data_ptr(),
                 None if dist is None else dist.data_ptr())


def _metric(m):
    return METRICS[m] if isinstance(m, str) else int(m)


def opts(keep_ratio=0.5, sample=10, delta=0.0, max_rounds=30, seed=0, precision="fp32",
         profile=False, balanced=False):
    o = Opts()
    load().knng_opts_default(ctypes.byref(o))
    o.keep_ratio = keep_ratio
    o.sample = sample
    o.delta = delta
    o.max_rounds = max_rounds
    o.seed = seed & (2 ** 64 - 1)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.flags = (FLAG_PROFILE if profile else 0) | (FLAG_BALANCED_APPEND if balanced else 0)
    return o


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _out(n, k, device):
    ids = torch.empty((n, k), dtype=torch.int32, device=device)
    dist = torch.empty((n, k), dtype=torch.float32, device=device)
    return ids, dist


def merge_workspace_size(n1, n2, d, k, kin1, kin2, metric="l2", **kw):
    o = opts(**kw)
    return load().knng_merge_workspace_size(n1, n2, d, k, kin1, kin2, _metric(metric),
                                            ctypes.byref(o))


def merge(S1, G1, S2, G2, k, metric="l2", stream=None, workspace=None, out=None, **kw):
    """S-Merge (knng_merge).  G1/G2 = (ids int32, dist fp32 or None), local ids.
    Returns (ids, dist, stats dict)."""
    lib = load()
    o = opts(**kw)
    s1, s2 = _set(S1), _set(S2)
    g1, g2 = _graph(*G1), _graph(*G2)
    n = S1.shape[0] + S2.shape[0]
    need = lib.knng_merge_workspace_size(S1.shape[0], S2.shape[0], S1.shape[1], k, g1.k, g2.k,
                                         _metric(metric), ctypes.byref(o))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=S1.device)
    ids, dist = out if out is not None else _out(n, k, S1.device)
    go = _graph(ids, dist)
    st = Stats()
    _check(lib.knng_merge(ctypes.byref(s1), ctypes.byref(g1), ctypes.byref(s2), ctypes.byref(g2),
                          k, _metric(metric), ctypes.byref(o), ctypes.byref(go),
                          _ptr(workspace), workspace.numel(), _stream(stream),
                          ctypes.byref(st)))
    return ids, dist, st.to_dict()


def merge_noalloc(S1, G1, S2, G2, k, metric="l2", stream=None, out=None, **kw):
    """S-Merge on the library's static scratch (knng_merge_noalloc): nothing
    is allocated on the device except `out` when it is not given.  Returns
    (ids, dist, stats dict)."""
    lib = load()
    o = opts(**kw)
    s1, s2 = _set(S1), _set(S2)
    g1, g2 = _graph(*G1), _graph(*G2)
    n = S1.shape[0] + S2.shape[0]
    ids, dist = out if out is not None else _out(n, k, S1.device)
    go = _graph(ids, dist)
    st = Stats()
    _check(lib.knng_merge_noalloc(ctypes.byref(s1), ctypes.byref(g1), ctypes.byref(s2),
                                  ctypes.byref(g2), k, _metric(metric), ctypes.byref(o),
                                  ctypes.byref(go), _stream(stream), ctypes.byref(st)))
    return ids, dist, st.to_dict()


def noalloc_scratch_bytes():
    return load().knng_merge_noalloc_scratch_bytes()


def expand(S, G, raw, k, metric="l2", stream=None, workspace=None, out=None, **kw):
    """J-Merge (knng_expand).  S may be None/empty (NN-Descent of raw).
    Returns (ids, dist, stats dict)."""
    lib = load()
    o = opts(**kw)
    d = raw.shape[1]
    if S is None or S.shape[0] == 0:
        s = Set(0, d, None)
        g = Graph(0, 0, None, None)
        nb, kin = 0, 0
    else:
        s = _set(S)
        g = _graph(*G)
        nb, kin = S.shape[0], g.k
    r = _set(raw)
    n = nb + raw.shape[0]
    need = lib.knng_expand_workspace_size(nb, raw.shape[0], d, k, kin, _metric(metric),
                                          ctypes.byref(o))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=raw.device)
    ids, dist = out if out is not None else _out(n, k, raw.device)
    go = _graph(ids, dist)
    st = Stats()
    _check(lib.knng_expand(ctypes.byref(s), ctypes.byref(g), ctypes.byref(r), k,
                           _metric(metric), ctypes.byref(o), ctypes.byref(go), _ptr(workspace),
                           workspace.numel(), _stream(stream), ctypes.byref(st)))
    return ids, dist, st.to_dict()


def merge_bruteforce(S1, G1, S2, G2, k, metric="l2", stream=None):
    """Brute-force cross merge (knng_merge_bruteforce).  Returns (ids, dist)."""
    lib = load()
    s1, s2 = _set(S1), _set(S2)
    g1, g2 = _graph(*G1), _graph(*G2)
    n = S1.shape[0] + S2.shape[0]
    need = lib.knng_bruteforce_workspace_size(S1.shape[0], S2.shape[0], S1.shape[1], k, g1.k,
                                              g2.k, _metric(metric))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=S1.device)
    ids, dist = _out(n, k, S1.device)
    go = _graph(ids, dist)
    _check(lib.knng_merge_bruteforce(ctypes.byref(s1), ctypes.byref(g1), ctypes.byref(s2),
                                     ctypes.byref(g2), k, _metric(metric), ctypes.byref(go),
                                     _ptr(ws), ws.numel(), _stream(stream)))
    return ids, dist


def exact_graph(S, k, metric="l2", stream=None):
    """Exact k-NN graph (knng_exact_graph).  Returns (ids, dist), local ids."""
    lib = load()
    s = _set(S)
    need = lib.knng_exact_graph_workspace_size(S.shape[0], S.shape[1], k, _metric(metric))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=S.device)
    ids, dist = _out(S.shape[0], k, S.device)
    go = _graph(ids, dist)
    _check(lib.knng_exact_graph(ctypes.byref(s), k, _metric(metric), ctypes.byref(go), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return ids, dist


def merge_tree(X, starts, graphs, k, metric="l2", stream=None, workspace=None, **kw):
    """Merge of consecutive row blocks of X by repeated S-Merge (knng_merge_tree).
    `starts`: nblocks+1 row offsets; `graphs`: per block (ids, dist or None),
    ids local to the block.  Returns (ids, dist, stats dict) over all of X."""
    lib = load()
    o = opts(**kw)
    xs = _set(X)
    nb = len(graphs)
    st_arr = (ctypes.c_int64 * (nb + 1))(*[int(v) for v in starts])
    garr = (Graph * nb)(*[_graph(*g) for g in graphs])
    kin_max = max(g[0].shape[1] for g in graphs)
    need = lib.knng_merge_tree_workspace_size(X.shape[0], X.shape[1], nb, st_arr, k, kin_max,
                                              _metric(metric), ctypes.byref(o))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    ids, dist = _out(X.shape[0], k, X.device)
    go = _graph(ids, dist)
    st = Stats()
    _check(lib.knng_merge_tree(ctypes.byref(xs), st_arr, garr, nb, k, _metric(metric),
                               ctypes.byref(o), ctypes.byref(go), _ptr(workspace),
                               workspace.numel(), _stream(stream), ctypes.byref(st)))
    d = st.to_dict()
    levels = [lvl for lvl in range(STATS_ROUNDS) if st.pairs[lvl]]
    d["level_evals"] = [st.updates[lvl] for lvl in levels]
    d["level_rounds"] = [st.pairs[lvl] for lvl in levels]
    d["level_ms"] = [st.gathered[lvl] / 1e3 for lvl in levels]
    return ids, dist, d


def hmerge(X, k, n_top, metric="l2", stream=None, workspace=None, **kw):
    """H-Merge (knng_hmerge): NN-Descent on n_top randomly chosen rows, then
    J-Merges that double the graph until it covers X.  Returns (ids, dist,
    stats dict with per-layer evaluations, rounds and wall times)."""
    lib = load()
    o = opts(**kw)
    xs = _set(X)
    need = lib.knng_hmerge_workspace_size(X.shape[0], X.shape[1], k, n_top, _metric(metric),
                                          ctypes.byref(o))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    ids, dist = _out(X.shape[0], k, X.device)
    go = _graph(ids, dist)
    st = Stats()
    _check(lib.knng_hmerge(ctypes.byref(xs), k, n_top, _metric(metric), ctypes.byref(o),
                           ctypes.byref(go), _ptr(workspace), workspace.numel(), _stream(stream),
                           ctypes.byref(st)))
    d = st.to_dict()
    layers = [lvl for lvl in range(STATS_ROUNDS) if st.pairs[lvl]]
    d["layer_evals"] = [st.updates[lvl] for lvl in layers]
    d["layer_rounds"] = [st.pairs[lvl] for lvl in layers]
    d["layer_ms"] = [st.gathered[lvl] / 1e3 for lvl in layers]
    return ids, dist, d


def hierarchy_shape(n, n_top, k):
    """[(rows, list size)] of the H-Merge layers, top first."""
    lib = load()
    L = lib.knng_hierarchy_shape(n, n_top, k, None, None, 0)
    rows = (ctypes.c_int64 * max(L, 1))()
    lists = (ctypes.c_int32 * max(L, 1))()
    lib.knng_hierarchy_shape(n, n_top, k, rows, lists, L)
    return [(rows[i], lists[i]) for i in range(L)]


def hmerge_hierarchy(X, k, n_top, metric="l2", stream=None, workspace=None, **kw):
    """H-Merge keeping its layers (knng_hmerge_hierarchy).  Returns (perm,
    xp, layers, stats): perm[i] = the row at position i, xp = X[perm], and
    layers[l] = (ids, dist) over positions, top layer first."""
    lib = load()
    o = opts(**kw)
    n, d = X.shape
    shape = hierarchy_shape(n, n_top, k)
    need = lib.knng_hmerge_workspace_size(n, d, k, n_top, _metric(metric), ctypes.byref(o))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    perm = torch.empty(n, dtype=torch.int32, device=X.device)
    xp = torch.empty((n, d), dtype=torch.float32, device=X.device)
    layers = [_out(r, kk, X.device) for r, kk in shape]
    gs = (Graph * len(layers))(*[_graph(i, dd) for i, dd in layers])
    st = Stats()
    _check(lib.knng_hmerge_hierarchy(ctypes.byref(_set(X)), k, n_top, _metric(metric),
                                     ctypes.byref(o), _ptr(perm), _ptr(xp), gs, len(layers),
                                     _ptr(workspace), workspace.numel(), _stream(stream),
                                     ctypes.byref(st)))
    return perm, xp, layers, st.to_dict()


def diversify(X, G, max_degree, metric="l2", stream=None):
    """Graph diversification (knng_diversify) of G = (ids, dist) over the rows
    of X.  Returns (ids, dist), max_degree columns."""
    lib = load()
    n, d = X.shape
    need = lib.knng_diversify_workspace_size(n, d, G[0].shape[1], _metric(metric))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    ids, dist = _out(n, max_degree, X.device)
    _check(lib.knng_diversify(ctypes.byref(_set(X)), ctypes.byref(_graph(*G)), max_degree,
                              _metric(metric), ctypes.byref(_graph(ids, dist)), _ptr(ws),
                              ws.numel(), _stream(stream)))
    return ids, dist


def search(X, layers, Q, topk, ef, seed=0, metric="l2", stream=None):
    """Top-down NN search (knng_search) of the rows of Q over layer graphs
    (ids tensors, or (ids, dist) pairs) over prefixes of X, top first.
    Returns (ids, dist, evals)."""
    lib = load()
    n, d = X.shape
    nq = Q.shape[0]
    need = lib.knng_search_workspace_size(n, d, nq, _metric(metric))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    ids_l = [L[0] if isinstance(L, (tuple, list)) else L for L in layers]
    gs = (Graph * len(ids_l))(*[Graph(t.shape[0], t.shape[1], t.data_ptr(), None)
                                for t in ids_l])
    for t in ids_l:
        assert t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()
    ids, dist = _out(nq, topk, X.device)
    ev = ctypes.c_int64()
    _check(lib.knng_search(ctypes.byref(_set(X)), gs, len(ids_l), ctypes.byref(_set(Q)), topk,
                           ef, seed & (2 ** 64 - 1), _metric(metric), _ptr(ids), _ptr(dist),
                           _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(ev)))
    return ids, dist, ev.value


def version():
    return load().knng_version()


class Server:
    """J-Merge serving (knng_server_*): a resident graph that absorbs requests
    of raw rows, each merged with the base independently, several at a time.
    base: device (n, d) fp32; G = (ids, dist or None) of the base, local ids.
    slots = 0 runs requests only inside step()."""

    def __init__(self, base, G, k, metric="l2", capacity=None, max_request=None, hbm_budget=0,
                 slots=4, batching=False, host_rounds=False, **kw):
        lib = load()
        o = opts(**kw)
        # the server reads base and G on its own streams (header: stream
        # contract); let the current stream's producers finish first
        torch.cuda.current_stream(base.device).synchronize()
        cfg = ServerConfig(int(capacity if capacity is not None else 2 * base.shape[0]),
                           int(max_request if max_request is not None else base.shape[0]),
                           int(hbm_budget), int(slots), int(bool(batching)),
                           int(bool(host_rounds)))
        h = ctypes.c_void_p()
        _check(lib.knng_server_create(ctypes.byref(_set(base)), ctypes.byref(_graph(*G)), k,
                                      _metric(metric), ctypes.byref(o), ctypes.byref(cfg),
                                      ctypes.byref(h)))
        self._h, self.k, self.d, self.device = h, k, base.shape[1], base.device
        self.slots = lib.knng_server_slots(h)

    def submit(self, raw, req_id):
        """Queues the rows of raw ((n, d) fp32, device tensor or host
        tensor/array; copied before return) as request req_id.  Returns the
        ticket."""
        if not isinstance(raw, torch.Tensor):
            raw = torch.from_numpy(raw)
        assert raw.dtype == torch.float32 and raw.dim() == 2 and raw.shape[1] == self.d
        raw = raw.contiguous()
        if raw.is_cuda:
            # read on the server's own stream (header: stream contract)
            torch.cuda.current_stream(raw.device).synchronize()
        t = ctypes.c_uint64()
        _check(load().knng_server_submit(self._h, ctypes.c_void_p(raw.data_ptr()), raw.shape[0],
                                         int(req_id) & (2 ** 64 - 1), ctypes.byref(t)))
        return t.value

    def step(self):
        """Servers without slots: runs the oldest queued request; False when
        none was queued."""
        ran = ctypes.c_int32()
        _check(load().knng_server_step(self._h, ctypes.byref(ran)))
        return bool(ran.value)

    def wait(self, ticket, n_rows, timeout_us=-1):
        """(ids, dist) host tensors of the request's rows and its info dict."""
        ids = torch.empty((n_rows, self.k), dtype=torch.int32)
        dist = torch.empty((n_rows, self.k), dtype=torch.float32)
        info = RequestInfo()
        _check(load().knng_server_wait(self._h, ticket, int(timeout_us),
                                       ctypes.c_void_p(ids.data_ptr()),
                                       ctypes.c_void_p(dist.data_ptr()), ctypes.byref(info)))
        return ids, dist, info.to_dict()

    def snapshot(self):
        """The resident graph as device tensors (ids, dist), rows sorted."""
        n = ctypes.c_int64()
        _check(load().knng_server_snapshot(self._h, None, ctypes.byref(n)))
        ids, dist = _out(n.value, self.k, self.device)
        g = _graph(ids, dist)
        _check(load().knng_server_snapshot(self._h, ctypes.byref(g), ctypes.byref(n)))
        return ids[:n.value], dist[:n.value]

    def fail_request(self, req_id):
        """Test hook: request req_id fails before its commit."""
        _check(load().knng_server_fail_request(self._h, int(req_id) & (2 ** 64 - 1)))

    def rebase(self):
        _check(load().knng_server_rebase(self._h))

    def status(self):
        b, c, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().knng_server_status(self._h, ctypes.byref(b), ctypes.byref(c),
                                         ctypes.byref(p)))
        return {"base": b.value, "committed": c.value, "pending": p.value}

    def close(self):
        if self._h:
            load().knng_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_bytes(capacity, max_request, d, k, kin, metric="l2", slots=1, **kw):
    o = opts(**kw)
    return load().knng_server_bytes(capacity, max_request, d, k, kin, _metric(metric),
                                    ctypes.byref(o), slots)
