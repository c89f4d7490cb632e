"""ctypes front end of the plain C oracle (knng_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  Nothing here is shared with, or imported
by, the HIP library or its Python binding.

Every function states the passage of Zhao et al., "On the Merge of k-NN
Graph", that it follows; the C file documents the canonical FP32 evaluation
order, the hash used for random draws and the readings of the paper taken
where it is silent.
"""
import ctypes
import os
import subprocess

import numpy as np

L2, COS, L1 = 0, 1, 2
METRICS = {"l2": L2, "cos": COS, "cosine": COS, "l1": L1}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knng_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

# -ffp-contract=off: the canonical FP32 order must not be fused by the compiler
BUILD_CMD = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-o", _LIB, _SRC, "-lm"]


def build():
    """Compile the oracle library (plain gcc, no GPU code)."""
    subprocess.run(BUILD_CMD, check=True)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("keep_ratio", ctypes.c_float), ("sample", ctypes.c_int32),
                ("delta", ctypes.c_float), ("max_rounds", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("evals", ctypes.c_int64),
                ("c", ctypes.c_int64 * 256), ("phi", ctypes.c_double * 257),
                ("pairs", ctypes.c_int64 * 256)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, I64, I32, F32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [ctypes.c_uint64]
        L.orc_hash.restype = ctypes.c_uint64
        L.orc_hash.argtypes = [ctypes.c_uint64] * 5
        L.orc_dist32.restype = F32
        L.orc_dist32.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
        L.orc_dist64.restype = ctypes.c_double
        L.orc_dist64.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
        L.orc_norm32.restype = F32
        L.orc_norm32.argtypes = [P, ctypes.c_int]
        L.orc_exact_graph.restype = ctypes.c_int
        L.orc_exact_graph.argtypes = [P, I64, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_merge_bruteforce.restype = ctypes.c_int
        L.orc_merge_bruteforce.argtypes = [P, I64, P, I64, ctypes.c_int, P, P, ctypes.c_int,
                                           P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_smerge.restype = ctypes.c_int
        L.orc_smerge.argtypes = [P, I64, P, I64, ctypes.c_int, P, P, ctypes.c_int, P, P,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(Params), P, P, ctypes.POINTER(Stats)]
        L.orc_jmerge.restype = ctypes.c_int
        L.orc_jmerge.argtypes = [P, I64, P, I64, ctypes.c_int, P, P, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int,
                                 P, P, ctypes.POINTER(Stats)]
        L.orc_draws.restype = None
        L.orc_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_uint32, I64, ctypes.c_int, P]
        L.orc_hmerge_order.restype = None
        L.orc_hmerge_order.argtypes = [ctypes.c_uint64, I64, P]
        L.orc_feistel4.restype = ctypes.c_uint64
        L.orc_feistel4.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        L.orc_diversify.restype = ctypes.c_int
        L.orc_diversify.argtypes = [P, I64, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                    ctypes.c_int, P, P]
        L.orc_search.restype = ctypes.c_int
        L.orc_search.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, I64,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_uint64, P, P,
                                 ctypes.POINTER(I64)]
        L.orc_dist64_rows.restype = None
        L.orc_dist64_rows.argtypes = [P, I64, ctypes.c_int, ctypes.c_int, P, I64, P]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _metric(m):
    return METRICS[m] if isinstance(m, str) else int(m)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: oracle returned {rc}")


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------

def splitmix64(state):
    """SplitMix64 output for generator state `state` (one step)."""
    return int(lib().orc_splitmix64(ctypes.c_uint64(state & (2**64 - 1))))


def hash5(seed, tag, a, b, c):
    """Chained SplitMix64 hash of a tuple (the draw stream of the merges)."""
    return int(lib().orc_hash(seed, tag, a, b, c))


TAG_APPEND, TAG_INIT, TAG_FWD, TAG_RNEW, TAG_ROLD = 0xA1, 0xA2, 0xB1, 0xB2, 0xB3
TAG_SEARCH = 0xD1


def draws(seed, tag, row, N, skip, m):
    """m distinct draws from [0, N) minus `skip` (-1: none), in draw order."""
    out = np.empty(m, np.int32)
    lib().orc_draws(seed, tag, row, N, skip, m, _ptr(out))
    return out


def dist32(metric, a, b):
    """Canonical FP32 distance (evaluation order in knng_oracle.c)."""
    a, b = _f32(a), _f32(b)
    return float(np.float32(lib().orc_dist32(_metric(metric), _ptr(a), _ptr(b), a.shape[0])))


def dist64(metric, a, b):
    """FP64 distance from the stored FP32 rows (plain definitions)."""
    a, b = _f32(a), _f32(b)
    return float(lib().orc_dist64(_metric(metric), _ptr(a), _ptr(b), a.shape[0]))


def norm32(a):
    a = _f32(a)
    return float(np.float32(lib().orc_norm32(_ptr(a), a.shape[0])))


# --------------------------------------------------------------------------
# graphs
# --------------------------------------------------------------------------

def exact_graph(X, k, metric="l2"):
    """Exact k-NN graph by brute force (Section 1): ids, canonical dists."""
    X = _f32(X)
    n, d = X.shape
    ids = np.empty((n, k), np.int32)
    dist = np.empty((n, k), np.float32)
    _check(lib().orc_exact_graph(_ptr(X), n, d, k, _metric(metric), _ptr(ids), _ptr(dist)),
           "exact_graph")
    return ids, dist


def merge_bruteforce(X1, G1, X2, G2, k, metric="l2"):
    """Brute-force cross merge (Section 1).  G1/G2 = (ids, dist or None)."""
    X1, X2 = _f32(X1), _f32(X2)
    n1, d = X1.shape
    n2 = X2.shape[0]
    g1i, g2i = _i32(G1[0]), _i32(G2[0])
    g1d = None if G1[1] is None else _f32(G1[1])
    g2d = None if G2[1] is None else _f32(G2[1])
    ids = np.empty((n1 + n2, k), np.int32)
    dist = np.empty((n1 + n2, k), np.float32)
    rc = lib().orc_merge_bruteforce(_ptr(X1), n1, _ptr(X2), n2, d, _ptr(g1i), _ptr(g1d),
                                    g1i.shape[1], _ptr(g2i), _ptr(g2d), g2i.shape[1], k,
                                    _metric(metric), _ptr(ids), _ptr(dist))
    _check(rc, "merge_bruteforce")
    return ids, dist


def _stats_dict(st):
    r = st.rounds
    m = min(r, 256)
    return {"rounds": r, "evals": int(st.evals), "c": [int(x) for x in st.c[:m]],
            "phi": [float(x) for x in st.phi[:m + 1]], "pairs": [int(x) for x in st.pairs[:m]]}


def _params(keep_ratio, sample, delta, max_rounds, seed):
    return Params(keep_ratio, sample, delta, max_rounds, seed & (2**64 - 1))


def smerge(X1, G1, X2, G2, k, metric="l2", keep_ratio=0.5, sample=10, delta=0.0,
           max_rounds=30, seed=0):
    """S-Merge, Algorithm 1.  Returns (ids, dist, stats)."""
    X1, X2 = _f32(X1), _f32(X2)
    n1, d = X1.shape
    n2 = X2.shape[0]
    g1i, g2i = _i32(G1[0]), _i32(G2[0])
    g1d = None if G1[1] is None else _f32(G1[1])
    g2d = None if G2[1] is None else _f32(G2[1])
    ids = np.empty((n1 + n2, k), np.int32)
    dist = np.empty((n1 + n2, k), np.float32)
    st = Stats()
    P = _params(keep_ratio, sample, delta, max_rounds, seed)
    rc = lib().orc_smerge(_ptr(X1), n1, _ptr(X2), n2, d, _ptr(g1i), _ptr(g1d), g1i.shape[1],
                          _ptr(g2i), _ptr(g2d), g2i.shape[1], k, _metric(metric),
                          ctypes.byref(P), _ptr(ids), _ptr(dist), ctypes.byref(st))
    _check(rc, "smerge")
    return ids, dist, _stats_dict(st)


def jmerge(Xb, G, Xr, k, metric="l2", keep_ratio=0.5, sample=10, delta=0.0, max_rounds=30,
           seed=0, balanced=False):
    """J-Merge, Algorithm 2 (G = (ids, dist or None) of the base set; the
    base set may be empty, which makes the call an NN-Descent build of Xr).
    balanced: only base rows selected with probability min(1, n_raw/n_base)
    take part in Divide and Append (identical to Algorithm 2 when
    n_raw >= n_base).  Returns (ids, dist, stats)."""
    Xr = _f32(Xr)
    nr, d = Xr.shape
    if Xb is None or len(Xb) == 0:
        Xb = np.zeros((0, d), np.float32)
        gi, gd, kin = None, None, 0
    else:
        Xb = _f32(Xb)
        gi = _i32(G[0])
        gd = None if G[1] is None else _f32(G[1])
        kin = gi.shape[1]
    nb = Xb.shape[0]
    ids = np.empty((nb + nr, k), np.int32)
    dist = np.empty((nb + nr, k), np.float32)
    st = Stats()
    P = _params(keep_ratio, sample, delta, max_rounds, seed)
    rc = lib().orc_jmerge(_ptr(Xb), nb, _ptr(Xr), nr, d, _ptr(gi), _ptr(gd), kin, k,
                          _metric(metric), ctypes.byref(P), int(bool(balanced)), _ptr(ids),
                          _ptr(dist), ctypes.byref(st))
    _check(rc, "jmerge")
    return ids, dist, _stats_dict(st)


def merge_tree(X, starts, graphs, k, metric="l2", **kw):
    """Many blocks merged by repeated S-Merge (Section 1: recursive two-graph
    merging; Section 3.1: sub-graphs merged pairwise).  Level by level the
    neighbouring row ranges (0,1), (2,3), ... are merged; an odd last range
    moves up unchanged.  Returns (ids, dist) over all rows of X."""
    X = _f32(X)
    segs = [(starts[b], starts[b + 1], graphs[b]) for b in range(len(graphs))]
    while len(segs) > 1:
        nxt = []
        for i in range(0, len(segs) - 1, 2):
            a, b, g1 = segs[i]
            _, c, g2 = segs[i + 1]
            ids, dist, _ = smerge(X[a:b], g1, X[b:c], g2, k, metric, **kw)
            nxt.append((a, c, (ids, dist)))
        if len(segs) % 2 == 1:
            a, c, g = segs[-1]
            nxt.append((a, c, (np.ascontiguousarray(g[0][:, :k]),
                               np.ascontiguousarray(g[1][:, :k]))))
        segs = nxt
    return segs[0][2]


def hmerge_order(seed, n):
    """Row at each position of H-Merge's random order (Section 3.3; the
    Feistel bijection documented in knng_oracle.c)."""
    out = np.empty(n, np.int32)
    lib().orc_hmerge_order(seed & (2**64 - 1), n, _ptr(out))
    return out


def feistel4(seed, x, h):
    """One pass of the 4-round Feistel network on 2h-bit values."""
    return int(lib().orc_feistel4(seed & (2**64 - 1), x, h))


def hmerge_layers(n, n_top, k):
    """(rows, list size) of every H-Merge layer, top first (Section 3.3): the
    first n_top rows, then doubling until n; k/2 entries above the bottom
    layer, k on it, never more than rows - 1."""
    rows = [min(n_top, n)]
    while rows[-1] < n:
        rows.append(min(2 * rows[-1], n))
    return [(m, min(k if m == n else k // 2, m - 1)) for m in rows]


def hmerge(X, k, n_top, metric="l2", keep_ratio=0.5, sample=10, delta=0.0, max_rounds=30,
           seed=0):
    """H-Merge, Section 3.3: NN-Descent builds the graph of a random subset of
    n_top rows; each later layer joins a raw random block as large as the
    current graph with J-Merge (Algorithm 2), until every row is in.  The
    rows are taken in the order hmerge_order(seed, n); layer l is seeded
    SplitMix64(seed ^ SplitMix64(l)).  Returns (ids, dist, per-layer stats)
    in the caller's row numbering, rows sorted by (distance, id)."""
    X = _f32(X)
    n = X.shape[0]
    order = hmerge_order(seed, n)
    Xp = X[order]
    ids = dist = None
    stats, below = [], 0
    for l, (rows, kk) in enumerate(hmerge_layers(n, n_top, k)):
        s_l = splitmix64(seed ^ splitmix64(l))
        base = Xp[:below] if below else None
        ids, dist, st = jmerge(base, (ids, dist), Xp[below:rows], kk, metric,
                               keep_ratio=keep_ratio, sample=sample, delta=delta,
                               max_rounds=max_rounds, seed=s_l)
        stats.append(st)
        below = rows
    # position i is row order[i]; ids are positions too
    rid = order[ids]
    srt = np.lexsort((rid, dist), axis=1)
    out_i = np.empty_like(rid)
    out_d = np.empty_like(dist)
    out_i[order] = np.take_along_axis(rid, srt, axis=1)
    out_d[order] = np.take_along_axis(dist, srt, axis=1)
    return out_i, out_d, stats


def hmerge_hierarchy(X, k, n_top, metric="l2", keep_ratio=0.5, sample=10, delta=0.0,
                     max_rounds=30, seed=0):
    """H-Merge (Section 3.3) keeping every layer: returns (order, layers),
    order[i] = the row at position i, layers[l] = (ids, dist) of layer l's
    graph over positions 0 .. rows_l - 1 (ids are positions), top layer
    first, exactly as hmerge builds them."""
    X = _f32(X)
    n = X.shape[0]
    order = hmerge_order(seed, n)
    Xp = X[order]
    ids = dist = None
    layers, below = [], 0
    for l, (rows, kk) in enumerate(hmerge_layers(n, n_top, k)):
        s_l = splitmix64(seed ^ splitmix64(l))
        base = Xp[:below] if below else None
        ids, dist, _ = jmerge(base, (ids, dist), Xp[below:rows], kk, metric,
                              keep_ratio=keep_ratio, sample=sample, delta=delta,
                              max_rounds=max_rounds, seed=s_l)
        layers.append((ids, dist))
        below = rows
    return order, layers


def diversify(X, G, max_deg, metric="l2"):
    """Graph diversification (Algorithm 3, Section 4) of G = (ids, dist) over
    the rows of X: Algorithm 3 on every list and on every reverse list, the
    two merged, the max_deg closest kept.  Returns (ids, dist)."""
    X = _f32(X)
    n, d = X.shape
    gi, gd = _i32(G[0]), _f32(G[1])
    k = gi.shape[1]
    ids = np.empty((n, max_deg), np.int32)
    dist = np.empty((n, max_deg), np.float32)
    _check(lib().orc_diversify(_ptr(X), n, d, _metric(metric), _ptr(gi), _ptr(gd), k, max_deg,
                               _ptr(ids), _ptr(dist)), "diversify")
    return ids, dist


def search(X, layers, Q, topk, ef, seed=0, metric="l2"):
    """Top-down NN search over a graph hierarchy (Section 4): layers[l] =
    ids (rows_l, deg_l) over the first rows_l rows of X, top layer first,
    the last layer holding every row.  Greedy descent on the upper layers
    from a seeded random top vertex, then a best-first search with a ranked
    list of ef entries on the bottom layer.  Returns (ids, dist, evals)."""
    X, Q = _f32(X), _f32(Q)
    d = X.shape[1]
    arrs = [_i32(a) for a in layers]
    nl = len(arrs)
    ptrs = (ctypes.c_void_p * nl)(*[a.ctypes.data for a in arrs])
    rows = np.array([a.shape[0] for a in arrs], np.int64)
    deg = np.array([a.shape[1] for a in arrs], np.int32)
    nq = Q.shape[0]
    ids = np.empty((nq, topk), np.int32)
    dist = np.empty((nq, topk), np.float32)
    ev = ctypes.c_int64()
    _check(lib().orc_search(_ptr(X), d, _metric(metric), ctypes.cast(ptrs, ctypes.c_void_p),
                            _ptr(rows), _ptr(deg), nl, _ptr(Q), nq, topk, ef,
                            seed & (2 ** 64 - 1), _ptr(ids), _ptr(dist), ctypes.byref(ev)),
           "search")
    return ids, dist, int(ev.value)


# --------------------------------------------------------------------------
# evaluation (Section 5.1)
# --------------------------------------------------------------------------

def dist64_rows(X, rows, metric="l2"):
    """FP64 distances (direct differences) of X[rows] to every row of X."""
    X = _f32(X)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], X.shape[0]), np.float64)
    lib().orc_dist64_rows(_ptr(X), X.shape[0], X.shape[1], _metric(metric), _ptr(rows),
                          rows.shape[0], _ptr(out))
    return out


def recall_at(ids, X, rows, k, metric="l2", D64=None):
    """recall@k of Eq. (recall) on the listed rows, tie-tolerant: an output
    neighbour counts as a true positive when its FP64 distance is within the
    exact k-th nearest distance of that row (self excluded).  Also returns
    the plain id-intersection form against one exact order.
    `D64` (optional) holds dist64_rows(X, rows, metric)."""
    rows = np.asarray(rows, dtype=np.int64)
    if D64 is None:
        D64 = dist64_rows(X, rows, metric)
    D = D64.copy()
    D[np.arange(rows.shape[0]), rows] = np.inf
    order = np.argsort(D, axis=1, kind="stable")[:, :k]
    kth = np.take_along_axis(D, order[:, k - 1:k], axis=1)[:, 0]
    hits_thr = 0
    hits_ids = 0
    for qi, r in enumerate(rows):
        out = ids[r, :k]
        valid = out[out >= 0]
        dv = D[qi, valid]
        hits_thr += int(np.sum(dv <= kth[qi]))
        hits_ids += len(np.intersect1d(valid, order[qi]))
    denom = rows.shape[0] * k
    return hits_thr / denom, hits_ids / denom


def phi(dist):
    """phi(G) of Eq. (1): the sum of all list distances."""
    d = np.asarray(dist, dtype=np.float64)
    return float(np.sum(d[np.isfinite(d)]))


def scanning_rate(evals, n):
    """Scanning rate of Eq. (scan): C / (n (n-1) / 2)."""
    return evals / (n * (n - 1) / 2.0)
