"""Thin Python binding of libann (ctypes).  Argument marshalling only: every
step runs in the library's HIP kernels; PyTorch supplies device memory and
streams.  The names mirror the C entry points of include/ann.h.

Importing this module loads libann.so and raises ImportError if it has not
been built (``python -m paper_2506_15986_amd.build``).  There is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libann.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libann.so is not built: run `python -m paper_2506_15986_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

ANN_OK, ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE, ANN_ENOTSUP = 0, 1, 2, 3, 4
ANN_FILTER_AUTO, ANN_FILTER_BITSET, ANN_FILTER_TAG16, ANN_FILTER_ID32, ANN_FILTER_TAG12 = 0, 1, 2, 3, 4
ANN_ORDER_WIDEST_FIRST, ANN_ORDER_AS_GIVEN = 0, 1
OP = dict(search=1, build_graph=2, gt_knn=3, select_hubs=4, entry_select=5, make_labels=6,
          hub_features=7, train_step=8)


class AnnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ann status %d: %s" % (status, msg))
        self.status = status


class ann_search_plan(ctypes.Structure):
    _fields_ = [("pool_cap", ctypes.c_int32), ("visited_log2", ctypes.c_int32),
                ("group", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("fp64", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("waves_per_query", ctypes.c_int32),
                ("query_order", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "ann_search_plan(%s)" % ", ".join("%s=%d" % kv for kv in self.as_dict().items())


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_F32 = ctypes.c_float
_F64 = ctypes.c_double


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_lib.ann_last_error.restype = ctypes.c_char_p
_lib.ann_version.restype = _I32
_sig("ann_workspace_size", _SZ, _I32, _I64, _I32, _I32, _I32)
_sig("ann_max_abs", _I32, _P, _I64, ctypes.POINTER(_F32), _P, _SZ, _P)
_sig("ann_default_plan", _I32, _I64, _I32, _I32, _I32, ctypes.POINTER(ann_search_plan))
_sig("ann_search", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _P, _I32, _P, _P, _I32, _P, _P, _P,
     _P, _I32, ctypes.POINTER(ann_search_plan), _P, _SZ, _P)


_sig("ann_search_noalloc", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _P, _I32, _P, _P, _I32, _P,
     _P, _P, _P, _I32, ctypes.POINTER(ann_search_plan), _P)
ANN_NOALLOC_MAX_QUERIES = 1 << 20


_sig("ann_gt_knn", _I32, _P, _I64, _I32, _P, _I32, _I32, _I32, _P, _P, _P, _SZ, _P)
_sig("ann_medoid", _I32, _P, _I64, _I32, ctypes.POINTER(_I32), _P, _SZ, _P)
_sig("ann_build_graph", _I32, _P, _I64, _I32, _I32, _I32, _F32, _P, ctypes.POINTER(_I32),
     ctypes.POINTER(_I32 * 2), _P, _SZ, _P)
_sig("ann_select_hubs", _I32, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _P, ctypes.POINTER(_I32),
     _P, _SZ, _P)
_sig("ann_hub_init_ids", _I32, _I64, _I32, ctypes.c_uint64, _P)
_sig("ann_hub_features", _I32, _P, _I64, _I32, _P, _I32, _I32, _P, _I32, _P, _P, _I32, _I32,
     _I32, _P, _P, _P, _SZ, _P)
_sig("ann_labels_workspace_size", _SZ, _I32, _I32, _I32)
_sig("ann_make_labels", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _P, _I32, _I32, _P, _I32, _P,
     _P, _I32, _P, _P, _P, _P, _SZ, _P)


class ann_tower(ctypes.Structure):
    _fields_ = [("din", _I32), ("hidden", _I32), ("dout", _I32), ("in_scale", _F32), ("W1", _P),
                ("b1", _P),
                ("W2", _P), ("b2", _P), ("W1b", _P), ("W2b", _P)]


class ann_tower_grads(ctypes.Structure):
    _fields_ = [("gW1", _P), ("gb1", _P), ("gW2", _P), ("gb2", _P)]


class ann_adam_state(ctypes.Structure):
    _fields_ = [(n, _P) for n in ("mW1", "vW1", "mb1", "vb1", "mW2", "vW2", "mb2", "vb2")]


class ann_entry_model(ctypes.Structure):
    _fields_ = [("query_tower", ann_tower), ("hub_emb", _P), ("hub_graph", _P), ("n_hubs", _I32),
                ("s", _I32), ("hub_ids", _P), ("hub_entry", _I32), ("medoid", _I32),
                ("L_h", _I32), ("theta", _F32), ("hub_plan", ann_search_plan)]


_sig("ann_hub_input", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _F32, _P, _P)
_sig("ann_tower_sync", _I32, ctypes.POINTER(ann_tower), _P)
_sig("ann_tower_workspace_size", _SZ, ctypes.POINTER(ann_tower), _I32)
_sig("ann_tower_forward", _I32, ctypes.POINTER(ann_tower), _P, _I32, _P, _P, _SZ, _P)
_sig("ann_train_workspace_size", _SZ, _I32, _I32, _I32, _I32, _I32, _I32)
_sig("ann_train_step", _I32, ctypes.POINTER(ann_tower), ctypes.POINTER(ann_tower),
     ctypes.POINTER(ann_tower_grads), ctypes.POINTER(ann_tower_grads),
     ctypes.POINTER(ann_adam_state), ctypes.POINTER(ann_adam_state), _P, _P, _I32, _P, _P, _I32,
     _F32, _F32, _I32, _P, _P, _P, _P, _P, _SZ, _P)
_sig("ann_navgraph_workspace_size", _SZ, _I32, _I32, _I32)
_sig("ann_navgraph_build", _I32, _P, _I32, _I32, _I32, _P, ctypes.POINTER(_I32), _P, _SZ, _P)
_sig("ann_entry_model_create", _I32, ctypes.POINTER(ann_entry_model),
     ctypes.POINTER(ctypes.POINTER(ann_entry_model)))
_sig("ann_entry_model_destroy", None, ctypes.POINTER(ann_entry_model))
_sig("ann_entry_workspace_size", _SZ, ctypes.POINTER(ann_entry_model), _I32)
_sig("ann_entry_select", _I32, ctypes.POINTER(ann_entry_model), _P, _I32, _I32, _P, _P, _P, _P,
     _SZ, _P)


def last_error() -> str:
    return _lib.ann_last_error().decode()


def version() -> int:
    return int(_lib.ann_version())


def _check(status):
    if status != ANN_OK:
        raise AnnError(status, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), \
        "expected a contiguous %s device tensor, got %s %s" % (dtype, t.dtype, t.device)
    return t


def workspace_size(op: str, n: int, dim: int, p0: int = 0, p1: int = 0) -> int:
    return int(_lib.ann_workspace_size(OP[op], n, dim, p0, p1))


def workspace(op: str, n: int, dim: int, p0: int = 0, p1: int = 0, device=None) -> torch.Tensor:
    nb = max(256, workspace_size(op, n, dim, p0, p1))
    return torch.empty(nb, dtype=torch.uint8, device=device or "cuda")


def default_plan(n: int, dim: int, R: int, L_max: int) -> ann_search_plan:
    p = ann_search_plan()
    _check(_lib.ann_default_plan(n, dim, R, L_max, ctypes.byref(p)))
    return p


def make_plan(**kw) -> ann_search_plan:
    p = ann_search_plan()
    for k, v in kw.items():
        setattr(p, k, int(v))
    return p


def ann_search(base: torch.Tensor, graph: torch.Tensor, queries: torch.Tensor,
               entry_ids: torch.Tensor | None, medoid: int, k, L, k_max: int | None = None,
               plan: ann_search_plan | None = None, want_stats: bool = True,
               trace_cap: int = 0, ws: torch.Tensor | None = None, out=None, stream=None):
    """Batched beam search.  k and L: ints or int32 device tensors (nq,).

    Returns (ids [nq,k_max] int32, dist [nq,k_max] float32 squared L2,
    stats [nq,4] int32 or None, trace [nq,trace_cap] int32 or None)."""
    _dev(base, torch.float32)
    _dev(graph, torch.int32)
    _dev(queries, torch.float32)
    n, dim = base.shape
    nq = queries.shape[0]
    R = graph.shape[1]
    dev = base.device
    if not torch.is_tensor(k):
        k = torch.full((nq,), int(k), dtype=torch.int32, device=dev)
    if not torch.is_tensor(L):
        L = torch.full((nq,), int(L), dtype=torch.int32, device=dev)
    if k_max is None:
        k_max = int(k.max().item()) if nq else 1
    if entry_ids is not None:
        _dev(entry_ids, torch.int32)
    if out is None:
        ids = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
        dist = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
        stats = torch.empty((nq, 4), dtype=torch.int32, device=dev) if want_stats else None
    else:
        ids, dist, stats = out
    trace = torch.empty((nq, trace_cap), dtype=torch.int32, device=dev) if trace_cap else None
    if ws is None:
        ws = workspace("search", n, dim, nq, 0, device=dev)
    _check(_lib.ann_search(_ptr(base), n, dim, _ptr(graph), R, _ptr(queries), nq,
                           _ptr(entry_ids), int(medoid), _ptr(k), _ptr(L), k_max, _ptr(ids),
                           _ptr(dist), _ptr(stats), _ptr(trace), int(trace_cap),
                           ctypes.byref(plan) if plan is not None else None,
                           _ptr(ws), ws.numel(), _stream(stream)))
    return ids, dist, stats, trace


_sig("ann_hub_search", _I32, _P, _I32, _I32, _P, _I32, _P, _I32, _I32, _I32, _P, _P, _P, _P, _I32,
     _P)


def ann_hub_search(emb: torch.Tensor, graph: torch.Tensor, qemb: torch.Tensor, start: int, L: int,
                   want_stats: bool = False, trace_cap: int = 0, stream=None):
    """Best-first search over the hub graph (k = 1, L <= 64, exact visited
    set).  Returns (best hub int32 [nq], its FP32 squared distance, stats
    [nq, 2] (distances, expansions) or None, trace [nq, trace_cap] or None)."""
    _dev(emb, torch.float32)
    _dev(graph, torch.int32)
    _dev(qemb, torch.float32)
    nh, dim = emb.shape
    nq = qemb.shape[0]
    dev = emb.device
    best = torch.empty(nq, dtype=torch.int32, device=dev)
    d2 = torch.empty(nq, dtype=torch.float32, device=dev)
    stats = torch.empty((nq, 2), dtype=torch.int32, device=dev) if want_stats else None
    trace = torch.empty((nq, trace_cap), dtype=torch.int32, device=dev) if trace_cap else None
    _check(_lib.ann_hub_search(_ptr(emb), nh, dim, _ptr(graph), graph.shape[1], _ptr(qemb), nq,
                               int(start), int(L), _ptr(best), _ptr(d2), _ptr(stats), _ptr(trace),
                               int(trace_cap), _stream(stream)))
    return best, d2, stats, trace


def ann_search_noalloc(base: torch.Tensor, graph: torch.Tensor, queries: torch.Tensor,
                       entry_ids: torch.Tensor | None, medoid: int, k: torch.Tensor,
                       L: torch.Tensor, k_max: int, out, plan: ann_search_plan | None = None,
                       trace=None, stream=None):
    """ann_search without a workspace: the library's fixed scratch array
    serves as the work counter and query order (at most
    ANN_NOALLOC_MAX_QUERIES queries).  k and L are int32 device tensors; the
    outputs (ids, dist, stats or None) are caller tensors, filled in place;
    trace is an int32 [nq, trace_cap] tensor or None.  Allocates nothing."""
    _dev(base, torch.float32)
    _dev(graph, torch.int32)
    _dev(queries, torch.float32)
    n, dim = base.shape
    nq = queries.shape[0]
    ids, dist, stats = out
    if entry_ids is not None:
        _dev(entry_ids, torch.int32)
    _check(_lib.ann_search_noalloc(_ptr(base), n, dim, _ptr(graph), graph.shape[1], _ptr(queries),
                                   nq, _ptr(entry_ids), int(medoid), _ptr(k), _ptr(L), int(k_max),
                                   _ptr(ids), _ptr(dist), _ptr(stats), _ptr(trace),
                                   int(trace.shape[1]) if trace is not None else 0,
                                   ctypes.byref(plan) if plan is not None else None,
                                   _stream(stream)))
    return ids, dist, stats


def ann_gt_knn(base: torch.Tensor, queries: torch.Tensor, k: int, exclude_self: bool = False,
               stream=None):
    """Exact top-k by (squared L2, id).  Returns (ids int32 [nq,k], dist float32)."""
    _dev(base, torch.float32)
    _dev(queries, torch.float32)
    n, dim = base.shape
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=base.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=base.device)
    ws = workspace("gt_knn", n, dim, nq, k, device=base.device)
    _check(_lib.ann_gt_knn(_ptr(base), n, dim, _ptr(queries), nq, k, int(exclude_self),
                           _ptr(ids), _ptr(dist), _ptr(ws), ws.numel(), _stream(stream)))
    return ids, dist


def ann_medoid(base: torch.Tensor, stream=None) -> int:
    _dev(base, torch.float32)
    n, dim = base.shape
    ws = workspace("build_graph", n, dim, 1, 3, device=base.device)
    m = _I32(-1)
    _check(_lib.ann_medoid(_ptr(base), n, dim, ctypes.byref(m), _ptr(ws), ws.numel(),
                           _stream(stream)))
    return int(m.value)


def ann_build_graph(base: torch.Tensor, knn_k: int, R: int, alpha: float, stream=None):
    """kNN -> alpha prune -> medoid -> repair.  Returns (graph int32 [n,R],
    medoid, (forward bridges, reverse bridges))."""
    _dev(base, torch.float32)
    n, dim = base.shape
    graph = torch.empty((n, R), dtype=torch.int32, device=base.device)
    ws = workspace("build_graph", n, dim, knn_k, R, device=base.device)
    m = _I32(-1)
    br = (_I32 * 2)()
    _check(_lib.ann_build_graph(_ptr(base), n, dim, knn_k, R, float(alpha), _ptr(graph),
                                ctypes.byref(m), ctypes.byref(br), _ptr(ws), ws.numel(),
                                _stream(stream)))
    del ws
    return graph, int(m.value), (int(br[0]), int(br[1]))


_sig("ann_build_graph_partitioned_workspace_size", _SZ, _I64, _I32, _I32, _I32, _I64, _I64)
_sig("ann_build_graph_partitioned", _I32, _P, _I64, _I32, _I32, _I32, _F32, _P, _I32, _I32, _P,
     ctypes.POINTER(_I32), ctypes.POINTER(_I32 * 2), _P, _SZ, _P)


def ann_build_graph_partitioned_workspace_size(n: int, dim: int, knn_k: int, R: int,
                                               max_members: int, max_home: int) -> int:
    return int(_lib.ann_build_graph_partitioned_workspace_size(n, dim, knn_k, R, max_members,
                                                               max_home))


_sig("ann_group_candidates_workspace_size", _SZ, _I32, _I32, _I64, _I64)
_sig("ann_group_candidates", _I32, _P, _I64, _I32, _I32, _P, _I32, _I32, _I32, _I32, _P, _P, _P,
     _SZ, _P)
_sig("ann_graph_from_candidates_workspace_size", _SZ, _I64, _I32, _I32)
_sig("ann_graph_from_candidates", _I32, _P, _I64, _I32, _P, _P, _I32, _I32, _F32, _P,
     ctypes.POINTER(_I32), ctypes.POINTER(_I32 * 2), _P, _SZ, _P)


def group_sizes(groups: np.ndarray, n_groups: int):
    """(members per group, home points per group) of an n x n_member label
    table (column 0 the home group, -1 = none, a repeated label counts once)."""
    g = np.asarray(groups).reshape(groups.shape[0], -1)
    home = np.bincount(g[:, 0], minlength=n_groups)
    first = np.ones(g.shape, bool)
    for c in range(1, g.shape[1]):
        first[:, c] = (g[:, c] >= 0) & (g[:, :c] != g[:, c:c + 1]).all(axis=1)
    mem = np.bincount(g[first], minlength=n_groups)
    return mem, home


def ann_build_graph_partitioned(base: torch.Tensor, knn_k: int, R: int, alpha: float,
                                groups: torch.Tensor, n_groups: int, stream=None):
    """kNN of each point among the members of its home group -> alpha prune
    -> medoid -> repair.  groups: n x n_member int32 (column 0 the home
    group).  Returns (graph int32 [n,R], medoid, (forward, reverse bridges))."""
    _dev(base, torch.float32)
    _dev(groups, torch.int32)
    n, dim = base.shape
    if groups.dim() == 1:
        groups = groups.reshape(n, 1)
    n_member = groups.shape[1]
    mem, home = group_sizes(groups.cpu().numpy(), n_groups)
    graph = torch.empty((n, R), dtype=torch.int32, device=base.device)
    nb = max(256, ann_build_graph_partitioned_workspace_size(n, dim, knn_k, R, int(mem.max()),
                                                             int(home.max())))
    ws = torch.empty(nb, dtype=torch.uint8, device=base.device)
    m = _I32(-1)
    br = (_I32 * 2)()
    _check(_lib.ann_build_graph_partitioned(_ptr(base), n, dim, knn_k, R, float(alpha),
                                            _ptr(groups), int(n_member), int(n_groups),
                                            _ptr(graph), ctypes.byref(m), ctypes.byref(br),
                                            _ptr(ws), ws.numel(), _stream(stream)))
    del ws
    return graph, int(m.value), (int(br[0]), int(br[1]))


def ann_group_candidates_workspace_size(dim: int, knn_k: int, max_members: int,
                                        max_home: int) -> int:
    return int(_lib.ann_group_candidates_workspace_size(dim, knn_k, max_members, max_home))


def ann_graph_from_candidates_workspace_size(n: int, dim: int, R: int) -> int:
    return int(_lib.ann_graph_from_candidates_workspace_size(n, dim, R))


def ann_group_candidates(base: torch.Tensor, knn_k: int, groups: torch.Tensor, n_groups: int,
                         g_begin: int, g_end: int, cand: torch.Tensor, cand_d2: torch.Tensor,
                         stream=None, sizes=None):
    """Candidate lists of the home points of groups [g_begin, g_end) written
    into cand (n x knn_k int32) / cand_d2 (n x knn_k float64).  sizes: the
    (members, homes) counts of group_sizes, when the caller has them."""
    _dev(base, torch.float32)
    _dev(groups, torch.int32)
    _dev(cand, torch.int32)
    _dev(cand_d2, torch.float64)
    n, dim = base.shape
    if groups.dim() == 1:
        groups = groups.reshape(n, 1)
    mem, home = sizes if sizes is not None else group_sizes(groups.cpu().numpy(), n_groups)
    nb = max(256, int(_lib.ann_group_candidates_workspace_size(dim, knn_k, int(mem.max()),
                                                               int(home.max()))))
    ws = torch.empty(nb, dtype=torch.uint8, device=base.device)
    _check(_lib.ann_group_candidates(_ptr(base), n, dim, knn_k, _ptr(groups), groups.shape[1],
                                     int(n_groups), int(g_begin), int(g_end), _ptr(cand),
                                     _ptr(cand_d2), _ptr(ws), ws.numel(), _stream(stream)))
    del ws


def ann_graph_from_candidates(base: torch.Tensor, cand: torch.Tensor, cand_d2: torch.Tensor,
                              R: int, alpha: float, stream=None):
    """alpha prune -> medoid -> repair of given candidate lists.  Returns
    (graph int32 [n,R], medoid, (forward, reverse bridges))."""
    _dev(base, torch.float32)
    _dev(cand, torch.int32)
    _dev(cand_d2, torch.float64)
    n, dim = base.shape
    graph = torch.empty((n, R), dtype=torch.int32, device=base.device)
    nb = max(256, int(_lib.ann_graph_from_candidates_workspace_size(n, dim, R)))
    ws = torch.empty(nb, dtype=torch.uint8, device=base.device)
    m = _I32(-1)
    br = (_I32 * 2)()
    _check(_lib.ann_graph_from_candidates(_ptr(base), n, dim, _ptr(cand), _ptr(cand_d2),
                                          cand.shape[1], R, float(alpha), _ptr(graph),
                                          ctypes.byref(m), ctypes.byref(br), _ptr(ws), ws.numel(),
                                          _stream(stream)))
    del ws
    return graph, int(m.value), (int(br[0]), int(br[1]))


_sig("ann_merge_candidates_workspace_size", _SZ)
_sig("ann_merge_candidates", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _P, _P, _P, _SZ, _P)


def ann_merge_candidates_workspace_size() -> int:
    return int(_lib.ann_merge_candidates_workspace_size())


def ann_merge_candidates(base: torch.Tensor, a_ids: torch.Tensor | None,
                         b_ids: torch.Tensor | None, stream=None):
    """Row-wise union of two id lists (n x a_w, n x b_w int32; either may be
    None), row i's own id and repeats dropped, ordered by (FP64 squared L2 to
    base row i, id).  Returns (ids int32, d2 float64), n x (a_w + b_w)."""
    _dev(base, torch.float32)
    n, dim = base.shape
    aw = bw = 0
    if a_ids is not None:
        _dev(a_ids, torch.int32)
        if a_ids.shape[0] != n:
            raise ValueError("a_ids must have one row per base point")
        aw = a_ids.shape[1]
    if b_ids is not None:
        _dev(b_ids, torch.int32)
        if b_ids.shape[0] != n:
            raise ValueError("b_ids must have one row per base point")
        bw = b_ids.shape[1]
    W = aw + bw
    ids = torch.empty((n, W), dtype=torch.int32, device=base.device)
    d2 = torch.empty((n, W), dtype=torch.float64, device=base.device)
    ws = torch.empty(max(256, ann_merge_candidates_workspace_size()), dtype=torch.uint8,
                     device=base.device)
    _check(_lib.ann_merge_candidates(_ptr(base), n, dim, _ptr(a_ids), aw, _ptr(b_ids), bw,
                                     _ptr(ids), _ptr(d2), _ptr(ws), ws.numel(), _stream(stream)))
    del ws
    return ids, d2


_sig("ann_select_hubs_hbkm_workspace_size", _SZ, _I64, _I32, _I32, _I32)
_sig("ann_select_hubs_hbkm", _I32, _P, _I64, _I32, _I32, _I32, ctypes.c_double, _I32, _P, _P, _P,
     _P, _SZ, _P)


def ann_select_hubs_hbkm_workspace_size(n: int, dim: int, k: int, levels: int) -> int:
    return int(_lib.ann_select_hubs_hbkm_workspace_size(n, dim, k, levels))


def ann_select_hubs_hbkm(base: torch.Tensor, k: int, levels: int, lam: float, iters: int,
                         stream=None):
    """Hierarchical balanced k-means (Algorithm 2) into k^levels clusters and
    their Definition 3 hubs.  Returns (hub_ids int32, centroids float64
    [k^levels, dim], assign int32 [n])."""
    _dev(base, torch.float32)
    n, dim = base.shape
    dev = base.device
    nc = k ** levels
    hub = torch.empty(nc, dtype=torch.int32, device=dev)
    cen = torch.empty((nc, dim), dtype=torch.float64, device=dev)
    asg = torch.empty(n, dtype=torch.int32, device=dev)
    nb = max(256, ann_select_hubs_hbkm_workspace_size(n, dim, k, levels))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(_lib.ann_select_hubs_hbkm(_ptr(base), n, dim, k, levels, float(lam), iters, _ptr(hub),
                                     _ptr(cen), _ptr(asg), _ptr(ws), ws.numel(), _stream(stream)))
    del ws
    return hub, cen, asg


def ann_hub_init_ids(n: int, n_hubs: int, seed: int) -> torch.Tensor:
    """The library's seeded k-means start: n_hubs distinct base ids (int32,
    host)."""
    out = torch.empty(n_hubs, dtype=torch.int32)
    _check(_lib.ann_hub_init_ids(n, n_hubs, seed & ((1 << 64) - 1), _ptr(out)))
    return out


def ann_select_hubs(base: torch.Tensor, n_hubs: int, iters: int,
                    init_ids: torch.Tensor | None = None, seed: int | None = None, stream=None):
    """Lloyd k-means + Definition 3 hubs from init_ids (device), or from the
    seeded start ann_hub_init_ids(n, n_hubs, seed).  Returns (hub_ids int32,
    centroids float64 [n_hubs, dim], assign int32 [n], steps)."""
    _dev(base, torch.float32)
    n, dim = base.shape
    dev = base.device
    if init_ids is None:
        if seed is None:
            raise ValueError("ann_select_hubs needs init_ids or a seed")
        init_ids = ann_hub_init_ids(n, n_hubs, seed).to(dev)
    _dev(init_ids, torch.int32)
    hub = torch.empty(n_hubs, dtype=torch.int32, device=dev)
    cen = torch.empty((n_hubs, dim), dtype=torch.float64, device=dev)
    asg = torch.empty(n, dtype=torch.int32, device=dev)
    steps = _I32(0)
    ws = workspace("select_hubs", n, dim, n_hubs, 0, device=dev)
    _check(_lib.ann_select_hubs(_ptr(base), n, dim, n_hubs, iters, _ptr(init_ids), _ptr(hub),
                                _ptr(cen), _ptr(asg), ctypes.byref(steps), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return hub, cen, asg, int(steps.value)


def ann_hub_features(base, graph, medoid: int, hub_ids, assign, centroids, h: int = 5,
                     wcap: int = 4096, standardise: bool = True, stream=None):
    """Returns (features float32 [n_hubs, 32], walk sizes int32 [n_hubs, 6])."""
    n, dim = base.shape
    nh = hub_ids.shape[0]
    R = graph.shape[1]
    dev = base.device
    f = torch.empty((nh, 32), dtype=torch.float32, device=dev)
    wsz = torch.empty((nh, 6), dtype=torch.int32, device=dev)
    ws = workspace("hub_features", n, dim, nh, R, device=dev)
    _check(_lib.ann_hub_features(_ptr(base), n, dim, _ptr(graph), R, int(medoid), _ptr(hub_ids),
                                 nh, _ptr(assign), _ptr(centroids), h, wcap, int(standardise),
                                 _ptr(f), _ptr(wsz), _ptr(ws), ws.numel(), _stream(stream)))
    return f, wsz


def ann_make_labels(base, graph, queries, truth, hits: int, cand_hubs, hub_ids, L_ladder,
                    want_table: bool = True, stream=None):
    """Returns (labels int32 [nq], table int32 [nq, M] or None, flags int32 [nq])."""
    n, dim = base.shape
    nq = queries.shape[0]
    dev = base.device
    M = cand_hubs.shape[1]
    kt = truth.shape[1]
    lad = (ctypes.c_int32 * len(L_ladder))(*[int(v) for v in L_ladder])
    labels = torch.empty(nq, dtype=torch.int32, device=dev)
    table = torch.empty((nq, M), dtype=torch.int32, device=dev) if want_table else None
    flags = torch.empty(nq, dtype=torch.int32, device=dev)
    nb = max(256, int(_lib.ann_labels_workspace_size(nq, M, kt)))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(_lib.ann_make_labels(_ptr(base), n, dim, _ptr(graph), graph.shape[1], _ptr(queries),
                                nq, _ptr(truth), kt, hits, _ptr(cand_hubs), M, _ptr(hub_ids),
                                lad, len(L_ladder), _ptr(labels), _ptr(table), _ptr(flags),
                                _ptr(ws), ws.numel(), _stream(stream)))
    return labels, table, flags


def ann_labels_workspace_size(nq: int, M: int, kt: int) -> int:
    return int(_lib.ann_labels_workspace_size(nq, M, kt))


class Tower:
    """Device-resident tower: FP32 masters, BF16 copies, gradients, Adam state."""

    def __init__(self, W1, b1, W2, b2, device="cuda", in_scale: float = 1.0):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        self.in_scale = float(in_scale)
        self.W1, self.b1, self.W2, self.b2 = f(W1), f(b1), f(W2), f(b2)
        self.hidden, self.din = self.W1.shape
        self.dout = self.W2.shape[0]
        self.W1b = torch.empty(self.W1.shape, dtype=torch.int16, device=device)
        self.W2b = torch.empty(self.W2.shape, dtype=torch.int16, device=device)
        self.g = [torch.zeros_like(t) for t in (self.W1, self.b1, self.W2, self.b2)]
        self.m = [torch.zeros_like(t) for t in (self.W1, self.b1, self.W2, self.b2)]
        self.v = [torch.zeros_like(t) for t in (self.W1, self.b1, self.W2, self.b2)]
        self.sync()

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2]

    def struct(self) -> ann_tower:
        return ann_tower(self.din, self.hidden, self.dout, self.in_scale, self.W1.data_ptr(),
                         self.b1.data_ptr(), self.W2.data_ptr(), self.b2.data_ptr(),
                         self.W1b.data_ptr(), self.W2b.data_ptr())

    def grads_struct(self) -> ann_tower_grads:
        return ann_tower_grads(*[t.data_ptr() for t in self.g])

    def adam_struct(self) -> ann_adam_state:
        m, v = self.m, self.v
        return ann_adam_state(m[0].data_ptr(), v[0].data_ptr(), m[1].data_ptr(), v[1].data_ptr(),
                              m[2].data_ptr(), v[2].data_ptr(), m[3].data_ptr(), v[3].data_ptr())

    def sync(self, stream=None):
        st = self.struct()
        _check(_lib.ann_tower_sync(ctypes.byref(st), _stream(stream)))

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        _dev(x, torch.float32)
        rows = x.shape[0]
        st = self.struct()
        out = torch.empty((rows, self.dout), dtype=torch.float32, device=x.device)
        nb = max(256, int(_lib.ann_tower_workspace_size(ctypes.byref(st), rows)))
        ws = torch.empty(nb, dtype=torch.uint8, device=x.device)
        _check(_lib.ann_tower_forward(ctypes.byref(st), _ptr(x), rows, _ptr(out), _ptr(ws), nb,
                                      _stream(stream)))
        return out


def ann_train_step(qt: Tower, ht: Tower, train_q, batch_idx, labels, hub_in, tau: float,
                   lr: float, step: int, ws=None, want_emb: bool = False, stream=None,
                   hub_in_grad=None):
    """One training step (step 0 = gradients only).  Returns (loss tensor,
    q_emb, h_emb) with the embeddings only when want_emb; hub_in_grad (a
    tensor shaped like hub_in) receives dL/d hub_in when given."""
    dev = train_q.device
    B = batch_idx.shape[0]
    nh = hub_in.shape[0]
    q_s, h_s = qt.struct(), ht.struct()
    qg, hg = qt.grads_struct(), ht.grads_struct()
    qa, ha = qt.adam_struct(), ht.adam_struct()
    nb = int(_lib.ann_train_workspace_size(B, nh, qt.din, ht.din, qt.hidden, qt.dout))
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    qe = torch.empty((B, qt.dout), dtype=torch.float32, device=dev) if want_emb else None
    he = torch.empty((nh, ht.dout), dtype=torch.float32, device=dev) if want_emb else None
    _check(_lib.ann_train_step(ctypes.byref(q_s), ctypes.byref(h_s), ctypes.byref(qg),
                               ctypes.byref(hg), ctypes.byref(qa), ctypes.byref(ha), _ptr(train_q),
                               _ptr(batch_idx), B, _ptr(labels), _ptr(hub_in), nh, float(tau),
                               float(lr), int(step), _ptr(loss), _ptr(qe), _ptr(he),
                               _ptr(hub_in_grad), _ptr(ws), ws.numel(), _stream(stream)))
    return loss, qe, he


_sig("ann_train_hub_workspace_size", _SZ, _I32, _I32, _I32, _I32, _I32, _I32, _I32)
_sig("ann_train_step_hub", _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I32, _I32, _I32, _P, _F32,
     _F32, _I32, _P, _P, _P, _P, _SZ, _P)
_sig("ann_hop_table_workspace_size", _SZ, _I64)
_sig("ann_hop_table", _I32, _P, _I64, _I32, _P, _I32, _P, _I64, _P, _P, _SZ, _P)


def ann_train_hub_workspace_size(hubs: int, P: int, N: int, din_q: int, din_h: int, hidden: int,
                                 dout: int) -> int:
    return int(_lib.ann_train_hub_workspace_size(hubs, P, N, din_q, din_h, hidden, dout))


def ann_train_step_hub(qt: Tower, ht: Tower, train_q, q_idx, hub_idx, P: int, N: int, hub_in,
                       tau: float, lr: float, step: int, ws=None, want_emb: bool = False,
                       stream=None):
    """One hub-anchored training step (Eq. 4 over Definition 4 queues;
    step 0 = gradients only).  q_idx: hubs x (P + N) query rows, positives
    first.  Returns (loss tensor, q_emb, h_emb)."""
    dev = train_q.device
    Bh = hub_idx.shape[0]
    rows = Bh * (P + N)
    assert q_idx.numel() == rows
    q_s, h_s = qt.struct(), ht.struct()
    qg, hg = qt.grads_struct(), ht.grads_struct()
    qa, ha = qt.adam_struct(), ht.adam_struct()
    nb = ann_train_hub_workspace_size(Bh, P, N, qt.din, ht.din, qt.hidden, qt.dout)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    qe = torch.empty((rows, qt.dout), dtype=torch.float32, device=dev) if want_emb else None
    he = torch.empty((Bh, ht.dout), dtype=torch.float32, device=dev) if want_emb else None
    _check(_lib.ann_train_step_hub(ctypes.byref(q_s), ctypes.byref(h_s), ctypes.byref(qg),
                                   ctypes.byref(hg), ctypes.byref(qa), ctypes.byref(ha),
                                   _ptr(train_q), _ptr(q_idx), _ptr(hub_idx), Bh, P, N,
                                   _ptr(hub_in), float(tau), float(lr), int(step), _ptr(loss),
                                   _ptr(qe), _ptr(he), _ptr(ws), ws.numel(), _stream(stream)))
    return loss, qe, he


def ann_hop_table_workspace_size(n: int) -> int:
    return int(_lib.ann_hop_table_workspace_size(n))



_sig("ann_make_queues_workspace_size", _SZ, _I64, _I32)
_sig("ann_make_queues", _I32, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _I64, _P, _I64,
     ctypes.POINTER(ctypes.c_int64), _P, _SZ, _P)


def ann_make_queues_workspace_size(nq: int, n_hubs: int) -> int:
    return int(_lib.ann_make_queues_workspace_size(nq, n_hubs))


def ann_make_queues(hops: torch.Tensor, t_pos: int, t_neg: int, stream=None):
    """Definition 4 queues from a hop table (nq x n_hubs uint8).  Returns
    (pos_off int64 [n_hubs+1], pos_q int32, neg_off, neg_q): queue h spans
    off[h]..off[h+1].  Two library calls: the first sizes the lists."""
    assert hops.is_cuda and hops.dtype == torch.uint8 and hops.is_contiguous()
    nq, nh = hops.shape
    dev = hops.device
    pos_off = torch.empty(nh + 1, dtype=torch.int64, device=dev)
    neg_off = torch.empty(nh + 1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(256, ann_make_queues_workspace_size(nq, nh)), dtype=torch.uint8,
                     device=dev)
    tot = (ctypes.c_int64 * 2)()
    pos_q = torch.empty(0, dtype=torch.int32, device=dev)
    neg_q = torch.empty(0, dtype=torch.int32, device=dev)
    for _ in range(2):
        st = _lib.ann_make_queues(_ptr(hops), nq, nh, int(t_pos), int(t_neg), _ptr(pos_off),
                                  _ptr(neg_off), _ptr(pos_q) if pos_q.numel() else None,
                                  pos_q.numel(), _ptr(neg_q) if neg_q.numel() else None,
                                  neg_q.numel(), tot, _ptr(ws), ws.numel(), _stream(stream))
        if st != ANN_ENOMEM:
            _check(st)
            break
        pos_q = torch.empty(int(tot[0]), dtype=torch.int32, device=dev)
        neg_q = torch.empty(int(tot[1]), dtype=torch.int32, device=dev)
    return pos_off, pos_q, neg_off, neg_q

def ann_hop_table(graph: torch.Tensor, hub_ids: torch.Tensor, targets: torch.Tensor, stream=None):
    """Definition 4 hop counts, uint8 [nq, n_hubs] (255: unreachable or
    farther than 254 hops)."""
    _dev(graph, torch.int32)
    _dev(hub_ids, torch.int32)
    _dev(targets, torch.int32)
    n, R = graph.shape
    nq, nh = targets.shape[0], hub_ids.shape[0]
    out = torch.empty((nq, nh), dtype=torch.uint8, device=graph.device)
    ws = torch.empty(max(256, ann_hop_table_workspace_size(n)), dtype=torch.uint8,
                     device=graph.device)
    _check(_lib.ann_hop_table(_ptr(graph), n, R, _ptr(hub_ids), nh, _ptr(targets), nq, _ptr(out),
                              _ptr(ws), ws.numel(), _stream(stream)))
    del ws
    return out


class ann_fusion(ctypes.Structure):
    _fields_ = [("heads", _I32), ("dk", _I32), ("dp", _I32), ("du", _I32), ("df", _I32),
                ("WQ", _P), ("WK", _P), ("WV", _P), ("WO", _P)]


_sig("ann_fusion_forward", _I32, ctypes.POINTER(ann_fusion), _P, _P, _P, _I32, _I32, _P, _P)
_sig("ann_fusion_workspace_size", _SZ, ctypes.POINTER(ann_fusion), _I32)
_sig("ann_fusion_backward", _I32, ctypes.POINTER(ann_fusion), _P, _P, _P, _I32, _I32, _P, _P, _P,
     _P, _P, _P, _SZ, _P)
_sig("ann_adam_step", _I32, _P, _P, _P, _P, _I64, _F32, _I32, _P)


def ann_adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                  lr: float, step: int, stream=None):
    _check(_lib.ann_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), float(lr),
                              int(step), _stream(stream)))


_sig("ann_fusion_tokens", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _F32, _P, _P, _P, _P)


def ann_fusion_tokens(base: torch.Tensor, graph: torch.Tensor, hub_ids: torch.Tensor,
                      scale: float, stream=None):
    """Fusion-embedding inputs per hub: (p [n_hubs, d], U [n_hubs, R, d],
    mask [n_hubs, R] uint8), from the hubs' vectors and graph neighbours."""
    _dev(base, torch.float32)
    _dev(graph, torch.int32)
    _dev(hub_ids, torch.int32)
    n, d = base.shape
    R = graph.shape[1]
    nh = hub_ids.shape[0]
    dev = base.device
    p = torch.empty((nh, d), dtype=torch.float32, device=dev)
    U = torch.empty((nh, R, d), dtype=torch.float32, device=dev)
    mask = torch.empty((nh, R), dtype=torch.uint8, device=dev)
    _check(_lib.ann_fusion_tokens(_ptr(base), n, d, _ptr(graph), R, _ptr(hub_ids), nh, float(scale),
                                  _ptr(p), _ptr(U), _ptr(mask), _stream(stream)))
    return p, U, mask


class Fusion:
    """Eq. 3 fusion embedding (ann_fusion_*): WQ, WK, WV [heads*dk x d],
    WO [df x heads*dk] on the device, with gradients and Adam moments."""

    def __init__(self, WQ, WK, WV, WO, heads: int, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()  # noqa: E731
        self.W = [f(WQ), f(WK), f(WV), f(WO)]
        self.heads = int(heads)
        self.dk = self.W[0].shape[0] // self.heads
        self.dp, self.du = self.W[0].shape[1], self.W[1].shape[1]
        self.df = self.W[3].shape[0]
        self.g = [torch.zeros_like(t) for t in self.W]
        self.m = [torch.zeros_like(t) for t in self.W]
        self.v = [torch.zeros_like(t) for t in self.W]

    def struct(self) -> ann_fusion:
        return ann_fusion(self.heads, self.dk, self.dp, self.du, self.df,
                          *[t.data_ptr() for t in self.W])

    def forward(self, p, U, mask, stream=None) -> torch.Tensor:
        nh, S = U.shape[0], U.shape[1]
        F = torch.empty((nh, self.df), dtype=torch.float32, device=p.device)
        st = self.struct()
        _check(_lib.ann_fusion_forward(ctypes.byref(st), _ptr(p), _ptr(U), _ptr(mask), nh, S,
                                       _ptr(F), _stream(stream)))
        return F

    def backward(self, p, U, mask, dF, stream=None):
        """Writes the four gradients into self.g."""
        nh, S = U.shape[0], U.shape[1]
        st = self.struct()
        nb = max(256, int(_lib.ann_fusion_workspace_size(ctypes.byref(st), nh)))
        ws = torch.empty(nb, dtype=torch.uint8, device=p.device)
        _check(_lib.ann_fusion_backward(ctypes.byref(st), _ptr(p), _ptr(U), _ptr(mask), nh, S,
                                        _ptr(dF), *[_ptr(t) for t in self.g], _ptr(ws), nb,
                                        _stream(stream)))

    def adam(self, lr: float, step: int, stream=None):
        for W, g, m, v in zip(self.W, self.g, self.m, self.v):
            ann_adam_step(W, g, m, v, lr, step, stream)


def ann_fusion_forward(fusion: Fusion, p, U, mask, stream=None) -> torch.Tensor:
    return fusion.forward(p, U, mask, stream)


def ann_fusion_backward(fusion: Fusion, p, U, mask, dF, stream=None):
    fusion.backward(p, U, mask, dF, stream)
    return fusion.g


def ann_fusion_workspace_size(fusion: Fusion, n_hubs: int) -> int:
    st = fusion.struct()
    return int(_lib.ann_fusion_workspace_size(ctypes.byref(st), n_hubs))


def ann_navgraph_build(hub_emb: torch.Tensor, s: int, stream=None):
    """Returns (hub graph int32 [n_hubs, s], hub entry index)."""
    _dev(hub_emb, torch.float32)
    nh, e = hub_emb.shape
    hg = torch.empty((nh, s), dtype=torch.int32, device=hub_emb.device)
    nb = int(_lib.ann_navgraph_workspace_size(nh, e, s))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=hub_emb.device)
    ent = _I32(-1)
    _check(_lib.ann_navgraph_build(_ptr(hub_emb), nh, e, s, _ptr(hg), ctypes.byref(ent), _ptr(ws),
                                   ws.numel(), _stream(stream)))
    return hg, int(ent.value)


class EntryModel:
    """The entry-selection model: query tower + hub embeddings + hub graph."""

    def __init__(self, qtower: Tower, hub_emb, hub_graph, hub_ids, hub_entry: int, medoid: int,
                 L_h: int = 32, theta: float = float("-inf"), hub_plan=None):
        self.qtower, self.hub_emb, self.hub_graph, self.hub_ids = qtower, hub_emb, hub_graph, hub_ids
        self.c = ann_entry_model(qtower.struct(), hub_emb.data_ptr(), hub_graph.data_ptr(),
                                 hub_emb.shape[0], hub_graph.shape[1], hub_ids.data_ptr(),
                                 int(hub_entry), int(medoid), int(L_h), float(theta),
                                 hub_plan if hub_plan is not None else ann_search_plan())
        self._ws = None

    def tune_L_h(self, sample_queries, agree: float = 0.995, ladder=(8, 12, 16, 24, 32, 48, 64)):
        """Smallest hub-search width whose best hub matches the exact nearest
        hub embedding (ann_gt_knn over the unit hub embeddings, i.e. the
        cosine argmax; a tie within 1e-6 in cosine counts as agreement) for at
        least `agree` of the sample queries.  Sets and returns it."""
        qe = self.qtower.forward(sample_queries)
        _, d2 = ann_gt_knn(self.hub_emb, qe, 1)
        best = 1.0 - 0.5 * d2[:, 0]
        choice, rates = int(ladder[-1]), []
        for L in ladder:
            self.c.L_h = int(L)
            self.c.hub_plan = ann_search_plan()
            _, sc, _ = ann_entry_select(self, sample_queries, want_score=True)
            ok = int(((sc - best).abs() <= 1e-6).sum().item()) / max(1, sc.shape[0])
            rates.append((int(L), round(ok, 5)))
            if ok >= agree:
                choice = int(L)
                break
        self.c.L_h = choice
        self.L_h_rates = rates
        return choice

    def tune_hub_plan(self, sample_queries, reps: int = 3):
        """Autotunes the hub-graph search on the embeddings of sample queries
        and keeps the fastest plan; returns it."""
        qe = self.qtower.forward(sample_queries)
        L = int(self.c.L_h)
        best, _ = ann_autotune_search(self.hub_emb, self.hub_graph, qe, None, int(self.c.hub_entry),
                                      1, L, 1, L, reps=reps)
        self.c.hub_plan = best
        return best

    def workspace(self, nq, device):
        nb = max(256, int(_lib.ann_entry_workspace_size(ctypes.byref(self.c), nq)))
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=device)
        return self._ws


def ann_entry_model_create(model: EntryModel):
    """A library handle: a checked host copy of the model's fields, its device
    pointers borrowed from `model` (keep `model` alive while it is used).
    Free it with ann_entry_model_destroy."""
    h = ctypes.POINTER(ann_entry_model)()
    _check(_lib.ann_entry_model_create(ctypes.byref(model.c), ctypes.byref(h)))
    return h


def ann_entry_model_destroy(handle) -> None:
    _lib.ann_entry_model_destroy(handle)


def ann_entry_select(model: EntryModel, queries: torch.Tensor, want_score: bool = False,
                     out=None, stream=None, handle=None):
    """Returns (entry ids int32 [nq], cosine float32 or None, best hub int32
    or None).  With `handle` (from ann_entry_model_create(model)) the library
    reads the model through it."""
    _dev(queries, torch.float32)
    nq, dim = queries.shape
    dev = queries.device
    ent = out if out is not None else torch.empty(nq, dtype=torch.int32, device=dev)
    sc = torch.empty(nq, dtype=torch.float32, device=dev) if want_score else None
    bh = torch.empty(nq, dtype=torch.int32, device=dev) if want_score else None
    ws = model.workspace(nq, dev)
    m = handle if handle is not None else ctypes.byref(model.c)
    _check(_lib.ann_entry_select(m, _ptr(queries), nq, dim, _ptr(ent), _ptr(sc), _ptr(bh),
                                 _ptr(ws), ws.numel(), _stream(stream)))
    return ent, sc, bh


def ann_tower_sync(tower: Tower, stream=None):
    tower.sync(stream)


def ann_tower_forward(tower: Tower, x: torch.Tensor, stream=None) -> torch.Tensor:
    return tower.forward(x, stream)


def ann_tower_workspace_size(tower: Tower, rows: int) -> int:
    st = tower.struct()
    return int(_lib.ann_tower_workspace_size(ctypes.byref(st), rows))


def ann_train_workspace_size(batch, n_hubs, din_q, din_h, hidden, dout) -> int:
    return int(_lib.ann_train_workspace_size(batch, n_hubs, din_q, din_h, hidden, dout))


def ann_entry_workspace_size(model: EntryModel, nq: int) -> int:
    return int(_lib.ann_entry_workspace_size(ctypes.byref(model.c), nq))


def ann_workspace_size(op: str, n: int, dim: int, p0: int = 0, p1: int = 0) -> int:
    return workspace_size(op, n, dim, p0, p1)


def ann_default_plan(n: int, dim: int, R: int, L_max: int) -> ann_search_plan:
    return default_plan(n, dim, R, L_max)


def ann_navgraph_workspace_size(n_hubs: int, dim: int, s: int) -> int:
    return int(_lib.ann_navgraph_workspace_size(n_hubs, dim, s))


def ann_hub_input(base: torch.Tensor, hub_ids: torch.Tensor, features: torch.Tensor | None = None,
                  vec_scale: float = 1.0, stream=None) -> torch.Tensor:
    """[base[hub_ids] * vec_scale | features] as an n_hubs x (dim + n_feat) FP32 matrix."""
    n, dim = base.shape
    nh = hub_ids.shape[0]
    nf = 0 if features is None else features.shape[1]
    out = torch.empty((nh, dim + nf), dtype=torch.float32, device=base.device)
    _check(_lib.ann_hub_input(_ptr(base), n, dim, _ptr(hub_ids), nh, _ptr(features), nf,
                              float(vec_scale), _ptr(out), _stream(stream)))
    return out


def ann_max_abs(x: torch.Tensor, stream=None) -> float:
    _dev(x, torch.float32)
    ws = torch.empty(256, dtype=torch.uint8, device=x.device)
    r = _F32(0)
    _check(_lib.ann_max_abs(_ptr(x), x.numel(), ctypes.byref(r), _ptr(ws), ws.numel(),
                            _stream(stream)))
    return float(r.value)


def input_scale(max_abs: float) -> float:
    """Power of two 2^-e with max_abs * 2^-e <= 1 (exact in BF16)."""
    import math
    if max_abs <= 0:
        return 1.0
    return 2.0 ** (-max(0, math.ceil(math.log2(max_abs))))


# ------------------------------------------------------------------ batch driver

class ann_query_batch(ctypes.Structure):
    _fields_ = [("base", _P), ("n", _I64), ("dim", _I32), ("graph", _P), ("R", _I32),
                ("queries", _P), ("nq", _I32), ("entry_ids", _P), ("medoid", _I32), ("k", _P),
                ("L", _P), ("k_max", _I32), ("out_ids", _P), ("out_dist", _P), ("stats", _P),
                ("plan", ann_search_plan), ("model", ctypes.POINTER(ann_entry_model)),
                ("entry_ws", _P), ("entry_ws_bytes", _SZ), ("search_ws", _P),
                ("search_ws_bytes", _SZ)]


ANN_STAGE_ENTRY, ANN_STAGE_SEARCH, ANN_STAGE_ALL = 1, 2, 3

_sig("ann_search_plan_lds", _SZ, ctypes.POINTER(ann_search_plan), _I64, _I32)
_sig("ann_autotune_candidates", _I32, _I64, _I32, _I32, _I32, ctypes.POINTER(ann_search_plan),
     _I32)
_sig("ann_autotune_workspace_size", _SZ, _I64, _I32, _I32, _I32)
_sig("ann_autotune_search", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _P, _I32, _P, _P, _I32, _P,
     _P, _P, ctypes.POINTER(ann_search_plan), _I32, _I32, ctypes.POINTER(ann_search_plan),
     ctypes.POINTER(_F32), _P, _SZ, _P)
_sig("ann_query_run", _I32, ctypes.POINTER(ann_query_batch), _I32, _P)
_sig("ann_query_graph_create", _I32, ctypes.POINTER(ann_query_batch), _I32,
     ctypes.POINTER(ctypes.c_void_p))
_sig("ann_query_graph_launch", _I32, ctypes.c_void_p, _P)
_lib.ann_query_graph_destroy.restype = None
_lib.ann_query_graph_destroy.argtypes = [ctypes.c_void_p]
_sig("ann_stream_create", _I32, ctypes.POINTER(ctypes.c_void_p))
_lib.ann_stream_destroy.restype = None
_lib.ann_stream_destroy.argtypes = [ctypes.c_void_p]


def ann_search_plan_lds(plan: ann_search_plan, n: int, dim: int) -> int:
    return int(_lib.ann_search_plan_lds(ctypes.byref(plan), n, dim))


def ann_autotune_candidates(n: int, dim: int, R: int, L_max: int) -> list:
    cnt = int(_lib.ann_autotune_candidates(n, dim, R, L_max, None, 0))
    arr = (ann_search_plan * max(cnt, 1))()
    _lib.ann_autotune_candidates(n, dim, R, L_max, arr, cnt)
    return [arr[i] for i in range(cnt)]


def ann_autotune_workspace_size(n: int, dim: int, nq: int, k_max: int) -> int:
    return int(_lib.ann_autotune_workspace_size(n, dim, nq, k_max))


def ann_autotune_search(base, graph, queries, entry_ids, medoid: int, k, L, k_max: int,
                        L_max: int, cands=None, reps: int = 3, stream=None):
    """Times the candidate plans on this batch; returns (best plan,
    [(plan, mean ms per launch or -1 when the plan does not fit)])."""
    n, dim = base.shape
    nq, R = queries.shape[0], graph.shape[1]
    dev = base.device
    if not torch.is_tensor(k):
        k = torch.full((nq,), int(k), dtype=torch.int32, device=dev)
    if not torch.is_tensor(L):
        L = torch.full((nq,), int(L), dtype=torch.int32, device=dev)
    if cands is None:
        cands = ann_autotune_candidates(n, dim, R, L_max)
    arr = (ann_search_plan * len(cands))(*cands)
    times = (_F32 * len(cands))()
    best = ann_search_plan()
    ids = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
    dist = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
    stats = torch.empty((nq, 4), dtype=torch.int32, device=dev)
    ws = torch.empty(max(256, ann_autotune_workspace_size(n, dim, nq, k_max)), dtype=torch.uint8,
                     device=dev)
    _check(_lib.ann_autotune_search(_ptr(base), n, dim, _ptr(graph), R, _ptr(queries), nq,
                                    _ptr(entry_ids), int(medoid), _ptr(k), _ptr(L), k_max,
                                    _ptr(ids), _ptr(dist), _ptr(stats), arr, len(cands), reps,
                                    ctypes.byref(best), times, _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return best, [(cands[i], float(times[i])) for i in range(len(cands))]


class QueryBatch:
    """Device buffers and the C description (ann_query_batch) of one batch of
    the query path; the tensors are kept alive with it."""

    def __init__(self, base, graph, medoid: int, queries, k, L, k_max: int, plan=None,
                 model: EntryModel | None = None, entry_ids=None, want_stats: bool = True):
        dev = base.device
        n, dim = base.shape
        nq, R = queries.shape[0], graph.shape[1]
        if not torch.is_tensor(k):
            k = torch.full((nq,), int(k), dtype=torch.int32, device=dev)
        if not torch.is_tensor(L):
            L = torch.full((nq,), int(L), dtype=torch.int32, device=dev)
        if plan is None:
            plan = default_plan(n, dim, R, int(L.max().item()) if nq else 1)
        if entry_ids is None and model is not None:
            entry_ids = torch.empty(nq, dtype=torch.int32, device=dev)
        self.base, self.graph, self.queries, self.k, self.L = base, graph, queries, k, L
        self.entry_ids, self.model, self.plan = entry_ids, model, plan
        self.ids = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
        self.dist = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
        self.stats = torch.empty((nq, 4), dtype=torch.int32, device=dev) if want_stats else None
        self.search_ws = workspace("search", n, dim, nq, device=dev)
        self.entry_ws = None
        self._model_c = None
        if model is not None:
            self._model_c = ann_entry_model.from_buffer_copy(model.c)
            nb = max(256, int(_lib.ann_entry_workspace_size(ctypes.byref(self._model_c), nq)))
            self.entry_ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.c = ann_query_batch(
            _ptr(base), n, dim, _ptr(graph), R, _ptr(queries), nq, _ptr(entry_ids), int(medoid),
            _ptr(k), _ptr(L), k_max, _ptr(self.ids), _ptr(self.dist), _ptr(self.stats), plan,
            ctypes.pointer(self._model_c) if self._model_c is not None else None,
            _ptr(self.entry_ws), self.entry_ws.numel() if self.entry_ws is not None else 0,
            _ptr(self.search_ws), self.search_ws.numel())

    def rebind(self, queries, k, L, entry_ids, ids, dist):
        """Points the batch at other rows of the same shape (device tensors
        whose row count is at most the one the workspaces were sized for):
        the queries, their k and L, the entry ids and the outputs."""
        nq = queries.shape[0]
        assert nq <= self.queries.shape[0], "rebind: more rows than the batch was sized for"
        for t in (queries, k, L, ids, dist) + ((entry_ids,) if entry_ids is not None else ()):
            assert t.is_cuda and t.is_contiguous()
        self.c.queries, self.c.k, self.c.L = _ptr(queries), _ptr(k), _ptr(L)
        self.c.entry_ids = _ptr(entry_ids) if entry_ids is not None else self.c.entry_ids
        self.c.out_ids, self.c.out_dist, self.c.stats = _ptr(ids), _ptr(dist), None
        self.c.nq = nq
        self._bound = (queries, k, L, entry_ids, ids, dist)     # kept alive with the batch

    def run(self, stages: int = ANN_STAGE_ALL, stream=None):
        _check(_lib.ann_query_run(ctypes.byref(self.c), stages, _stream(stream)))
        return self.ids, self.dist, self.stats

    def graph_exec(self, stages: int = ANN_STAGE_ALL) -> "QueryGraph":
        return QueryGraph(self, stages)


class QueryGraph:
    """A HIP graph of a QueryBatch's stages (ann_query_graph_*)."""

    def __init__(self, batch: QueryBatch, stages: int = ANN_STAGE_ALL):
        self.batch = batch
        h = ctypes.c_void_p()
        _check(_lib.ann_query_graph_create(ctypes.byref(batch.c), stages, ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(_lib.ann_query_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            _lib.ann_query_graph_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ann_query_run(batch: QueryBatch, stages: int = ANN_STAGE_ALL, stream=None):
    return batch.run(stages, stream)


def ann_query_graph_create(batch: QueryBatch, stages: int = ANN_STAGE_ALL) -> QueryGraph:
    return QueryGraph(batch, stages)


def ann_query_graph_launch(graph: QueryGraph, stream=None):
    graph.launch(stream)


def ann_query_graph_destroy(graph: QueryGraph):
    graph.close()


def ann_stream_create(device=None) -> torch.cuda.ExternalStream:
    """A stream with a hardware queue of its own (ann_stream_create), as a
    torch stream.  The HIP stream lives until ann_stream_destroy; nothing
    destroys it implicitly (not at garbage collection, not at exit)."""
    h = ctypes.c_void_p()
    with torch.cuda.device(device if device is not None else torch.cuda.current_device()):
        _check(_lib.ann_stream_create(ctypes.byref(h)))
        return torch.cuda.ExternalStream(h.value)


def ann_stream_destroy(stream: torch.cuda.ExternalStream):
    """Destroys a stream from ann_stream_create (waits for its pending work)."""
    _lib.ann_stream_destroy(ctypes.c_void_p(stream.cuda_stream))


_DEDICATED: dict = {}


def dedicated_stream(i: int, device=None) -> torch.cuda.ExternalStream:
    """Stream i of a per-device set made by ann_stream_create on first use and
    kept for the life of the process, so that repeated pipelines and servers
    reuse the same hardware queues instead of asking for new ones."""
    dv = torch.device(device if device is not None else torch.cuda.current_device())
    key = (dv.index if dv.index is not None else torch.cuda.current_device(), int(i))
    if key not in _DEDICATED:
        _DEDICATED[key] = ann_stream_create(key[0])
    return _DEDICATED[key]
