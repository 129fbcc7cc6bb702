"""Thin Python binding of libann (ctypes).  Argument marshalling only: every
step runs in the library's HIP kernels; PyTorch supplies device memory and
streams.  The names mirror the C entry points of include/ann.h.

Importing this module loads libann.so and raises ImportError if it has not
been built (``python -m paper_2506_15986_amd.build``).  There is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libann.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libann.so is not built: run `python -m paper_2506_15986_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

ANN_OK, ANN_EINVAL, ANN_ENOMEM, ANN_EDEVICE, ANN_ENOTSUP = 0, 1, 2, 3, 4
OP = dict(search=1, build_graph=2, gt_knn=3, select_hubs=4, entry_select=5, make_labels=6,
          hub_features=7, train_step=8)


class AnnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ann status %d: %s" % (status, msg))
        self.status = status


class ann_search_plan(ctypes.Structure):
    _fields_ = [("pool_cap", ctypes.c_int32), ("visited_log2", ctypes.c_int32),
                ("group", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("fp64", ctypes.c_int32)]

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
_sig("ann_default_plan", _I32, _I64, _I32, _I32, _I32, ctypes.POINTER(ann_search_plan))
_sig("ann_search", _I32, _P, _I64, _I32, _P, _I32, _P, _I32, _P, _I32, _P, _P, _I32, _P, _P, _P,
     _P, _I32, ctypes.POINTER(ann_search_plan), _P, _SZ, _P)


_sig("ann_gt_knn", _I32, _P, _I64, _I32, _P, _I32, _I32, _I32, _P, _P, _P, _SZ, _P)
_sig("ann_medoid", _I32, _P, _I64, _I32, ctypes.POINTER(_I32), _P, _SZ, _P)
_sig("ann_build_graph", _I32, _P, _I64, _I32, _I32, _I32, _F32, _P, ctypes.POINTER(_I32),
     ctypes.POINTER(_I32 * 2), _P, _SZ, _P)
_sig("ann_select_hubs", _I32, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _P, ctypes.POINTER(_I32),
     _P, _SZ, _P)
_sig("ann_hub_features", _I32, _P, _I64, _I32, _P, _I32, _I32, _P, _I32, _P, _P, _I32, _I32,
     _I32, _P, _P, _P, _SZ, _P)


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


def ann_select_hubs(base: torch.Tensor, n_hubs: int, iters: int, init_ids: torch.Tensor,
                    stream=None):
    """Lloyd k-means + Definition 3 hubs.  Returns (hub_ids int32, centroids
    float64 [n_hubs, dim], assign int32 [n], steps)."""
    _dev(base, torch.float32)
    _dev(init_ids, torch.int32)
    n, dim = base.shape
    dev = base.device
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
