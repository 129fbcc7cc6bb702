"""CPU oracle for the GATE search path — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import this package.  The product library never does; the two
share no code.  Everything here is plain FP64 arithmetic written for a reader
to check against the paper by eye:

* ``oracle.c`` (ctypes below): distances, exact kNN, alpha pruning, medoid,
  connectivity repair, best-first beam search (Algorithm 1), Lloyd k-means hubs
  (Definition 3), hub navigation graph and entry selection (high-tier graph
  section), label search.
* ``towers.py``: the two-tower model, InfoNCE loss (Eq. 2 / Eq. 4 reading) and
  Adam, in NumPy float64.
* ``features.py``: the 32 per-hub topology features (guided-walk sampling).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        _lib = ctypes.CDLL(LIB)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F32 = ctypes.c_float
_F64 = ctypes.c_double


def _declare(L):
    L.oracle_sqdist.argtypes = [_P, _P, ctypes.c_int]
    L.oracle_sqdist.restype = _F64
    L.oracle_knn.argtypes = [_P, _I64, ctypes.c_int, _P, _I64, ctypes.c_int, ctypes.c_int, _P, _P]
    L.oracle_alpha_prune.argtypes = [_P, _I64, ctypes.c_int, _P, _P, ctypes.c_int, ctypes.c_int, _F32, _P]
    L.oracle_medoid.argtypes = [_P, _I64, ctypes.c_int]
    L.oracle_medoid.restype = _I32
    L.oracle_repair.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _I32, _P, _P]
    L.oracle_search.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _P, _I64, _P, _P, _P,
                                ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_int,
                                ctypes.c_int, _P, ctypes.c_int]
    L.oracle_kmeans_hubs.argtypes = [_P, _I64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P,
                                     _P, _P, _P]
    L.oracle_kmeans_hubs.restype = ctypes.c_int
    L.oracle_hub_graph.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P]
    L.oracle_hub_medoid.argtypes = [_P, ctypes.c_int, ctypes.c_int]
    L.oracle_hub_medoid.restype = _I32
    L.oracle_hub_features.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _I32, _P,
                                      ctypes.c_int, _P, _P, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _P, _P]
    L.oracle_entry_select.argtypes = [_P, _I64, _P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int,
                                      _P, _I32, ctypes.c_int, _F64, _I32, _P, _P, _P]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# --------------------------------------------------------------------------
def sqdist(x, y) -> float:
    x, y = _f32(x), _f32(y)
    return lib().oracle_sqdist(_ptr(x), _ptr(y), x.shape[-1])


def knn(base, queries, k: int, exclude_self: bool = False):
    """Exact k nearest neighbours by (d2, id).  Returns (ids int32, d2 float64)."""
    base, queries = _f32(base), _f32(queries)
    nq = queries.shape[0]
    ids = np.empty((nq, k), np.int32)
    dd = np.empty((nq, k), np.float64)
    lib().oracle_knn(_ptr(base), base.shape[0], base.shape[1], _ptr(queries), nq, k,
                     int(exclude_self), _ptr(ids), _ptr(dd))
    return ids, dd


def alpha_prune(base, cand, cand_d2, R: int, alpha: float):
    base = _f32(base)
    cand = _i32(cand)
    cand_d2 = np.ascontiguousarray(cand_d2, np.float64)
    n = base.shape[0]
    g = np.empty((n, R), np.int32)
    lib().oracle_alpha_prune(_ptr(base), n, base.shape[1], _ptr(cand), _ptr(cand_d2),
                             cand.shape[1], R, _F32(alpha), _ptr(g))
    return g


def medoid(base) -> int:
    base = _f32(base)
    return int(lib().oracle_medoid(_ptr(base), base.shape[0], base.shape[1]))


def repair(base, graph, med: int):
    """Returns (repaired copy of graph, n_forward, n_reverse)."""
    base = _f32(base)
    g = _i32(graph).copy()
    nf = _I32(0)
    nr = _I32(0)
    lib().oracle_repair(_ptr(base), base.shape[0], base.shape[1], _ptr(g), g.shape[1],
                        int(med), ctypes.byref(nf), ctypes.byref(nr))
    return g, nf.value, nr.value


def build_graph(base, knn_k: int, R: int, alpha: float):
    """kNN(knn_k) -> alpha prune to R-2 -> medoid -> repair.

    Returns (graph, medoid, n_forward, n_reverse, cand_ids, cand_d2)."""
    cand, cd2 = knn(base, base, knn_k, exclude_self=True)
    g = alpha_prune(base, cand, cd2, R, alpha)
    m = medoid(base)
    g, nf, nr = repair(base, g, m)
    return g, m, nf, nr, cand, cd2


def search(base, graph, queries, entry, k, L, k_max: int | None = None,
           trace_cap: int = 0, truth=None, c_hit: int = 0, want_visited: bool = False,
           threads: int = 0):
    """Best-first beam search (Algorithm 1 reading).

    k and L may be scalars or per-query arrays.  Returns a dict with ids
    (nq x k_max, -1 padded), d2 (float64, +inf padded), ndc, hops, ndc_hit,
    trace (nq x trace_cap) and visited (nq x n uint8) when asked for."""
    base, queries = _f32(base), _f32(queries)
    graph = _i32(graph)
    n, d = base.shape
    nq = queries.shape[0]
    entry = _i32(np.broadcast_to(np.asarray(entry), (nq,)))
    kk = _i32(np.broadcast_to(np.asarray(k), (nq,)))
    LL = _i32(np.broadcast_to(np.asarray(L), (nq,)))
    if k_max is None:
        k_max = int(kk.max())
    ids = np.empty((nq, k_max), np.int32)
    dd = np.empty((nq, k_max), np.float64)
    stats = np.empty((nq, 3), np.int64)
    trace = np.empty((nq, trace_cap), np.int32) if trace_cap > 0 else None
    kt = 0
    if truth is not None:
        truth = _i32(truth)
        kt = truth.shape[1]
    vis = np.zeros((nq, n), np.uint8) if want_visited else None
    lib().oracle_search(_ptr(base), n, d, _ptr(graph), graph.shape[1], _ptr(queries), nq,
                        _ptr(entry), _ptr(kk), _ptr(LL), k_max, _ptr(ids), _ptr(dd),
                        _ptr(stats), _ptr(trace), trace_cap, _ptr(truth), kt, c_hit,
                        _ptr(vis), threads)
    out = dict(ids=ids, d2=dd, ndc=stats[:, 0], hops=stats[:, 1], ndc_hit=stats[:, 2])
    if trace is not None:
        out["trace"] = trace
    if vis is not None:
        out["visited"] = vis
    return out


def kmeans_hubs(base, n_hubs: int, iters: int, init_ids):
    """Lloyd k-means from the given initial centroids, then Definition 3 hubs.

    Returns dict(hub_ids, centroids (float64), assign, steps, objective)."""
    base = _f32(base)
    init_ids = _i32(init_ids)
    n, d = base.shape
    hub = np.empty(n_hubs, np.int32)
    cen = np.empty((n_hubs, d), np.float64)
    asg = np.empty(n, np.int32)
    obj = np.full(iters, np.nan)
    steps = lib().oracle_kmeans_hubs(_ptr(base), n, d, n_hubs, iters, _ptr(init_ids),
                                     _ptr(hub), _ptr(cen), _ptr(asg), _ptr(obj))
    return dict(hub_ids=hub, centroids=cen, assign=asg, steps=steps, objective=obj[:steps])


def hub_graph(emb, s: int):
    emb = _f32(emb)
    nh, e = emb.shape
    hg = np.empty((nh, s), np.int32)
    lib().oracle_hub_graph(_ptr(emb), nh, e, s, _ptr(hg))
    return hg


def hub_medoid(emb) -> int:
    emb = _f32(emb)
    return int(lib().oracle_hub_medoid(_ptr(emb), emb.shape[0], emb.shape[1]))


def entry_select(qemb, hemb, hg, hub_ids, Lh: int, theta: float, med: int,
                 hub_entry: int | None = None):
    """Search the hub graph for each query embedding; returns (entry_ids,
    score (cosine, float64), best hub index)."""
    qemb, hemb = _f32(qemb), _f32(hemb)
    hg, hub_ids = _i32(hg), _i32(hub_ids)
    nq, e = qemb.shape
    nh = hemb.shape[0]
    if hub_entry is None:
        hub_entry = hub_medoid(hemb)
    ent = np.empty(nq, np.int32)
    sc = np.empty(nq, np.float64)
    bh = np.empty(nq, np.int32)
    lib().oracle_entry_select(_ptr(qemb), nq, _ptr(hemb), nh, e, _ptr(hg), hg.shape[1],
                              _ptr(hub_ids), int(hub_entry), Lh, float(theta), int(med),
                              _ptr(ent), _ptr(sc), _ptr(bh))
    return ent, sc, bh


def hub_features(base, graph, med: int, hub_ids, assign, centroids, h: int = 5,
                 wcap: int = 4096, standardize: bool = True):
    """32 topology features per hub from a guided walk (see oracle.c).
    Returns (features nh x 32 float64, walk node counts per depth nh x 6)."""
    base = _f32(base)
    graph = _i32(graph)
    hub_ids = _i32(hub_ids)
    assign = _i32(assign)
    centroids = np.ascontiguousarray(centroids, np.float64)
    nh = hub_ids.shape[0]
    f = np.empty((nh, 32), np.float64)
    ws = np.empty((nh, 6), np.int32)
    lib().oracle_hub_features(_ptr(base), base.shape[0], base.shape[1], _ptr(graph), graph.shape[1],
                              int(med), _ptr(hub_ids), nh, _ptr(assign), _ptr(centroids), h, wcap,
                              int(standardize), _ptr(f), _ptr(ws))
    return f, ws


def recall(found_ids, truth_ids, k: int) -> np.ndarray:
    """recall@k = |R ∩ R'| / k per query (Eq. 1)."""
    f = np.asarray(found_ids)[:, :k]
    t = np.asarray(truth_ids)[:, :k]
    hits = np.array([len(set(a[a >= 0].tolist()) & set(b.tolist())) for a, b in zip(f, t)])
    return hits / float(k)


def make_labels(base, graph, train_q, truth, cand_hubs, hub_ids, L_lab: int, c_hit: int,
                threads: int = 0):
    """Per training query: the candidate hub whose search reaches c_hit of the
    true neighbours with the fewest distance computations (ties: smaller hub
    index).  cand_hubs holds hub indices (nq x M) ordered nearest first; when
    no candidate reaches c_hit the label is the first candidate.  Returns
    (label hub index, ndc_hit table nq x M with -1 for never)."""
    nq, M = cand_hubs.shape
    table = np.empty((nq, M), np.int64)
    for m in range(M):
        ent = np.asarray(hub_ids)[cand_hubs[:, m]]
        r = search(base, graph, train_q, ent, 1, L_lab, truth=truth, c_hit=c_hit,
                   threads=threads)
        table[:, m] = r["ndc_hit"]
    label = np.empty(nq, np.int32)
    for i in range(nq):
        best = None
        for m in range(M):
            if table[i, m] < 0:
                continue
            cand = (int(table[i, m]), int(cand_hubs[i, m]))
            if best is None or cand < best:
                best = cand
        # no candidate reached c_hit: fall back to the nearest candidate hub
        label[i] = best[1] if best is not None else int(cand_hubs[i, 0])
    return label, table
