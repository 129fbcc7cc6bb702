"""CPU oracle for the GATE search path — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import this package.  The product library never does; the two
share no code.  Everything here is plain FP64 arithmetic written for a reader
to check against the paper by eye:

* ``oracle.c`` (ctypes below): distances, exact kNN, alpha pruning, medoid,
  connectivity repair, best-first beam search (Algorithm 1), Lloyd k-means hubs
  (Definition 3), label search, hub topology features.
* hub navigation graph and entry selection (high-tier graph section) are
  composed below from kNN, medoid and search on the unit hub embeddings.
* ``towers.py``: the two-tower model, InfoNCE loss (Eq. 2 / Eq. 4 reading) and
  Adam, in NumPy float64.
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
    L.oracle_repair.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _I32, _P, ctypes.c_int,
                                _P, _P]
    L.oracle_search.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _P, _I64, _P, _P, _P,
                                ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_int]
    L.oracle_kmeans_hubs.argtypes = [_P, _I64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P,
                                     _P, _P, _P]
    L.oracle_kmeans_hubs.restype = ctypes.c_int
    L.oracle_hop_table.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _P, _I64, _P]
    L.oracle_hbkm.argtypes = [_P, _I64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _F64,
                              ctypes.c_int, _P, _P, _P]
    L.oracle_hub_features.argtypes = [_P, _I64, ctypes.c_int, _P, ctypes.c_int, _I32, _P,
                                      ctypes.c_int, _P, _P, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _P, _P]


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


def repair(base, graph, med: int, cand=None):
    """Returns (repaired copy of graph, n_forward, n_reverse).  With candidate
    lists, each bridge is the first eligible entry of the unreached point's
    list when there is one (the same node as the argmin when the lists are
    the global nearest neighbours)."""
    base = _f32(base)
    g = _i32(graph).copy()
    nf = _I32(0)
    nr = _I32(0)
    c = None if cand is None else _i32(cand)
    lib().oracle_repair(_ptr(base), base.shape[0], base.shape[1], _ptr(g), g.shape[1],
                        int(med), _ptr(c), 0 if c is None else c.shape[1], ctypes.byref(nf),
                        ctypes.byref(nr))
    return g, nf.value, nr.value


def build_graph(base, knn_k: int, R: int, alpha: float):
    """kNN(knn_k) -> alpha prune to R-2 -> medoid -> repair.

    Returns (graph, medoid, n_forward, n_reverse, cand_ids, cand_d2)."""
    cand, cd2 = knn(base, base, knn_k, exclude_self=True)
    g = alpha_prune(base, cand, cd2, R, alpha)
    m = medoid(base)
    g, nf, nr = repair(base, g, m)
    return g, m, nf, nr, cand, cd2


def knn_in_home_group(base, groups, k: int):
    """Candidate lists restricted to overlapping groups (a construction
    shortcut for large indexes; the paper assumes the proximity graph is
    given).  groups is n x m: row p lists p's groups, column 0 its home
    group, -1 = none.  The list of p holds the k nearest by (d2, id) among
    the points q != p whose row lists p's home group; -1 / +inf padded.
    Returns (ids int32, d2 float64)."""
    base = _f32(base)
    groups = np.asarray(groups).reshape(base.shape[0], -1)
    n = base.shape[0]
    ids = np.full((n, k), -1, np.int32)
    dd = np.full((n, k), np.inf)
    for g in np.unique(groups[:, 0]):
        mem = np.flatnonzero((groups == g).any(axis=1)).astype(np.int32)
        home = np.flatnonzero(groups[:, 0] == g)
        kk = min(k + 1, len(mem))
        li, ld = knn(base[mem], base[home], kk)
        for r, p in enumerate(home):
            keep = mem[li[r]] != p
            got = mem[li[r][keep]][:k]
            ids[p, :len(got)] = got
            dd[p, :len(got)] = ld[r][keep][:k]
    return ids, dd


def build_graph_grouped(base, groups, knn_k: int, R: int, alpha: float):
    """build_graph with the candidate lists of knn_in_home_group; repair
    bridges from those lists first (full argmin only when none is eligible).
    Returns (graph, medoid, n_forward, n_reverse, cand_ids, cand_d2)."""
    cand, cd2 = knn_in_home_group(base, groups, knn_k)
    g = alpha_prune(base, cand, cd2, R, alpha)
    m = medoid(base)
    g, nf, nr = repair(base, g, m, cand)
    return g, m, nf, nr, cand, cd2


def merge_candidates(pool_ids, pool_d2, knn_ids, knn_d2):
    """Row-wise union of two candidate lists (the point's own search pool and
    its exact kNN list), point i's own id dropped, duplicates once, ordered by
    (d2, id); -1 / +inf padded to the two widths together."""
    n = pool_ids.shape[0]
    W = pool_ids.shape[1] + knn_ids.shape[1]
    ids = np.full((n, W), -1, np.int32)
    dd = np.full((n, W), np.inf)
    for i in range(n):
        seen = {}
        for a, b in ((pool_ids[i], pool_d2[i]), (knn_ids[i], knn_d2[i])):
            for c, v in zip(a.tolist(), b.tolist()):
                if c >= 0 and c != i:
                    seen[c] = v
        items = sorted((v, c) for c, v in seen.items())
        ids[i, :len(items)] = [c for _, c in items]
        dd[i, :len(items)] = [v for v, _ in items]
    return ids, dd


def build_graph_nsg(base, knn_k: int, L: int, R: int, path: int = 0):
    """NSG-style graph: exact kNN(knn_k); each point searched for from the
    medoid on the kNN graph's first min(knn_k, 64) columns with beam width L;
    its pool, and with path > 0 also the first `path` nodes that search
    expanded, merged with its kNN list (merge_candidates); pruning at
    alpha = 1 to R - 2; repair with bridges from the merged lists first.
    Returns (graph, medoid, n_forward, n_reverse, cand_ids, cand_d2)."""
    base = _f32(base)
    cand, cd2 = knn(base, base, knn_k, exclude_self=True)
    m = medoid(base)
    g0 = np.ascontiguousarray(cand[:, :min(knn_k, 64)])
    res = search(base, g0, base, m, L, L, trace_cap=path)
    a_ids, a_d2 = res["ids"], res["d2"]
    if path > 0:
        tr = res["trace"]
        td2 = np.array([[sqdist(base[i], base[c]) if c >= 0 else np.inf for c in tr[i]]
                        for i in range(tr.shape[0])])
        a_ids = np.concatenate([a_ids, tr], 1)
        a_d2 = np.concatenate([a_d2, td2], 1)
    ids, dd = merge_candidates(a_ids, a_d2, cand, cd2)
    g = alpha_prune(base, ids, dd, R, 1.0)
    g, nf, nr = repair(base, g, m, ids)
    return g, m, nf, nr, ids, dd


def search(base, graph, queries, entry, k, L, k_max: int | None = None,
           trace_cap: int = 0, want_visited: bool = False, threads: int = 0):
    """Best-first beam search (Algorithm 1 reading).

    k and L may be scalars or per-query arrays.  Returns a dict with ids
    (nq x k_max, -1 padded), d2 (float64, +inf padded), ndc, hops, trace
    (nq x trace_cap) and visited (nq x n uint8) when asked for."""
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
    stats = np.empty((nq, 2), np.int64)
    trace = np.empty((nq, trace_cap), np.int32) if trace_cap > 0 else None
    vis = np.zeros((nq, n), np.uint8) if want_visited else None
    lib().oracle_search(_ptr(base), n, d, _ptr(graph), graph.shape[1], _ptr(queries), nq,
                        _ptr(entry), _ptr(kk), _ptr(LL), k_max, _ptr(ids), _ptr(dd),
                        _ptr(stats), _ptr(trace), trace_cap, _ptr(vis), threads)
    out = dict(ids=ids, d2=dd, ndc=stats[:, 0], hops=stats[:, 1])
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


_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, count: int):
    """The first `count` outputs of SplitMix64 (Steele, Lea and Flood, "Fast
    splittable pseudorandom number generators", OOPSLA 2014) started from the
    64-bit state `seed`: each draw adds the golden-ratio increment
    0x9E3779B97F4A7C15 to the state and returns the new state through the
    generator's finaliser (two xor-shift-multiply rounds and a last xor-shift)."""
    out = []
    state = seed & _MASK64
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out.append(z ^ (z >> 31))
    return out


def floyd_sample(n: int, m: int, draw):
    """m distinct values out of 0..n-1 by Robert Floyd's algorithm (Bentley
    and Floyd, "Programming pearls: a sample of brilliance", CACM 1987): for
    j = n - m, ..., n - 1 draw t uniformly from 0..j (draw(j)) and take t, or
    j when t was taken already.  Returns the values in the order taken."""
    taken, seen = [], set()
    for j in range(n - m, n):
        t = draw(j)
        v = j if t in seen else t
        seen.add(v)
        taken.append(v)
    return taken


def hub_init_ids(n: int, n_hubs: int, seed: int):
    """Seeded initial centroids for kmeans_hubs (the paper leaves the k-means
    start open): Floyd's sampling of n_hubs base ids, its i-th draw from
    0..j being floor(x_i * (j + 1) / 2^64) for the i-th SplitMix64 output x_i
    (the multiply-shift map of Lemire, "Fast random integer generation in an
    interval", 2019, without its rejection step)."""
    xs = iter(splitmix64(seed, n_hubs))
    return np.array(floyd_sample(n, n_hubs, lambda j: (next(xs) * (j + 1)) >> 64), np.int32)


def hbkm_hubs(base, k: int, levels: int, lam: float, iters: int):
    """Hierarchical balanced k-means (Algorithm 2) into k^levels clusters,
    then Definition 3 hubs.  Returns dict(hub_ids, centroids (float64),
    assign)."""
    base = _f32(base)
    n, d = base.shape
    nc = k ** levels
    hub = np.empty(nc, np.int32)
    cen = np.empty((nc, d), np.float64)
    asg = np.empty(n, np.int32)
    lib().oracle_hbkm(_ptr(base), n, d, k, levels, float(lam), iters, _ptr(asg), _ptr(cen),
                      _ptr(hub))
    return dict(hub_ids=hub, centroids=cen, assign=asg)


def hop_table(graph, hub_ids, targets):
    """Definition 4 hop counts: H[q, h] = shortest-path length along the
    graph's edges from hub h to targets[q] (the query's nearest neighbour);
    255 when unreachable or more than 254 hops.  uint8 [nq, nh]."""
    graph = _i32(graph)
    hub_ids, targets = _i32(hub_ids), _i32(targets)
    out = np.empty((targets.shape[0], hub_ids.shape[0]), np.uint8)
    lib().oracle_hop_table(_ptr(graph), graph.shape[0], graph.shape[1], _ptr(hub_ids),
                           hub_ids.shape[0], _ptr(targets), targets.shape[0], _ptr(out))
    return out


def sample_queues(H, t_pos: int, t_neg: int):
    """Positive and negative queries of every hub (Definition 4): with m_h
    the smallest hop count any query has from hub h, q is positive for h when
    H[q, h] <= m_h + t_pos and negative when H[q, h] >= m_h + t_neg (the
    negatives' "analogous" definition read with t_neg; unreachable counts as
    far).  Hubs no query reaches have neither.  Returns two lists of int64
    query-index arrays, one entry per hub."""
    H = np.asarray(H)
    pos, neg = [], []
    for h in range(H.shape[1]):
        col = H[:, h].astype(np.int64)
        reach = col < 255
        if not reach.any():
            pos.append(np.zeros(0, np.int64))
            neg.append(np.zeros(0, np.int64))
            continue
        m = col[reach].min()
        pos.append(np.flatnonzero(reach & (col <= m + t_pos)))
        neg.append(np.flatnonzero(~reach | (col >= m + t_neg)))
    return pos, neg


def hub_graph(emb, s: int):
    """Navigation graph over hubs (high-tier graph section): row i = the s hubs
    of largest cosine with hub i, self excluded.  The embeddings are unit
    vectors, so |e_i - e_j|^2 = 2 - 2 cos(e_i, e_j): the cosine order is the
    order by squared L2 distance, ties by index."""
    ids, _ = knn(emb, emb, s, exclude_self=True)
    return ids


def hub_medoid(emb) -> int:
    """Where the hub-graph search starts: the hub of largest cosine with the
    mean embedding direction.  For unit rows, argmax <h, mu> = argmin
    |h - mu|^2, i.e. the medoid of the embeddings."""
    return medoid(emb)


def entry_select(qemb, hemb, hg, hub_ids, Lh: int, theta: float, med: int,
                 hub_entry: int | None = None):
    """Entry points: beam search (width Lh) over the hub graph from the hub
    entry by squared L2 between unit embeddings (the cosine order); the best
    hub h has cos = 1 - d2/2; entry = hub_ids[h], or the medoid when
    cos < theta.  Returns (entry_ids, cos (float64), best hub index)."""
    if hub_entry is None:
        hub_entry = hub_medoid(hemb)
    r = search(hemb, hg, qemb, int(hub_entry), 1, Lh)
    bh = r["ids"][:, 0].astype(np.int32)
    cos = 1.0 - 0.5 * r["d2"][:, 0]
    ent = np.where(cos < theta, np.int32(med), np.asarray(hub_ids, np.int32)[bh]).astype(np.int32)
    return ent, cos, bh


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


def make_labels(base, graph, train_q, truth, cand_hubs, hub_ids, L_ladder, hits: int,
                threads: int = 0):
    """Training labels (stand-in for the paper's hop-count queues, same intent:
    which hub serves a query best).  For query i and candidate hub m the beam
    search runs from hub_ids[cand_hubs[i, m]] with each width of L_ladder
    (increasing); cost(i, m) = ndc of the first width whose top-kt holds at
    least `hits` of truth[i] (kt = truth.shape[1]), -1 if none does.  The
    label is the candidate of least cost, ties to the smaller hub index, else
    the first candidate.  Returns (labels, cost table nq x M)."""
    truth = np.asarray(truth)
    nq, M = cand_hubs.shape
    kt = truth.shape[1]
    table = np.full((nq, M), -1, np.int64)
    for m in range(M):
        ent = np.asarray(hub_ids)[cand_hubs[:, m]]
        for L in L_ladder:
            r = search(base, graph, train_q, ent, kt, int(L), threads=threads)
            for i in range(nq):
                if table[i, m] >= 0:
                    continue
                h = len(set(r["ids"][i].tolist()) & set(truth[i].tolist()))
                if h >= hits:
                    table[i, m] = r["ndc"][i]
    label = np.empty(nq, np.int32)
    for i in range(nq):
        best = None
        for m in range(M):
            if table[i, m] < 0:
                continue
            cand = (int(table[i, m]), int(cand_hubs[i, m]))
            if best is None or cand < best:
                best = cand
        label[i] = best[1] if best is not None else int(cand_hubs[i, 0])
    return label, table
