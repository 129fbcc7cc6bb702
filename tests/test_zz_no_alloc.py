"""ann_search_noalloc (the search with the library's fixed scratch array in
place of a workspace) against ann_search on the same inputs, on two calls in
a row, the second with a smaller batch: ids, distances and statistics must be
identical (same kernels, same plan), and agree with the oracle."""
import numpy as np
import pytest
import torch

import oracle
from tests.common import int_index, say

pytestmark = pytest.mark.gpu


def _ann():
    from paper_2506_15986_amd import ann
    return ann


def _run_both(ann, bd, gd, qd, ed, med, kk, LL, k_max, plan):
    nq = qd.shape[0]
    dev = bd.device
    ref = ann.ann_search(bd, gd, qd, ed, med, kk, LL, k_max=k_max, plan=plan)
    out = (torch.full((nq, k_max), -7, dtype=torch.int32, device=dev),
           torch.full((nq, k_max), -7.0, dtype=torch.float32, device=dev),
           torch.full((nq, 4), -7, dtype=torch.int32, device=dev))
    got = ann.ann_search_noalloc(bd, gd, qd, ed, med, kk, LL, k_max, out, plan=plan)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref[:3]], [t.cpu().numpy() for t in got]


@pytest.mark.parametrize("wpq", [1, 2])
def test_noalloc_search_equals_workspace_search_twice(wpq):
    ann = _ann()
    say("case: ann_search_noalloc vs ann_search, 20k x 128 integers, waves per query %d" % wpq)
    ix = int_index()
    dev = torch.device("cuda:0")
    base, q, g, med = ix["base"], ix["q"], ix["graph"], ix["medoid"]
    bd, gd, qd = (torch.from_numpy(base).to(dev), torch.from_numpy(g).to(dev),
                  torch.from_numpy(q).to(dev))
    nq = q.shape[0]
    r = np.random.default_rng(40 + wpq)
    ent = r.integers(0, base.shape[0], nq).astype(np.int32)
    ks = r.choice([1, 5, 10], nq).astype(np.int32)
    Ls = np.maximum(ks, r.choice([16, 48, 96], nq)).astype(np.int32)
    plan = ann.default_plan(base.shape[0], base.shape[1], g.shape[1], 96)
    plan.waves_per_query = wpq
    plan.waves_per_block = wpq
    plan.group = 16 if wpq > 1 else plan.group
    assert plan.query_order == ann.ANN_ORDER_WIDEST_FIRST    # the order lives in the scratch
    ed = torch.from_numpy(ent).to(dev)
    kk, LL = torch.from_numpy(ks).to(dev), torch.from_numpy(Ls).to(dev)
    ref, got = _run_both(ann, bd, gd, qd, ed, med, kk, LL, 10, plan)
    for a, b in zip(ref, got):
        assert (a == b).all()
    o = oracle.search(base, g, q, ent, ks, Ls, k_max=10)
    assert (got[0] == o["ids"]).all()
    assert (got[1].astype(np.float64)[got[0] >= 0] == o["d2"][got[0] >= 0]).all()
    assert (got[2][:, 2] == o["hops"]).all()
    say("case: second call, smaller batch (37 queries), other widths and entries")
    m = 37
    ent2 = np.full(m, med, np.int32)
    Ls2 = np.full(m, 24, np.int32)
    ks2 = np.full(m, 10, np.int32)
    ref2, got2 = _run_both(ann, bd, gd, qd[:m].contiguous(), torch.from_numpy(ent2).to(dev), med,
                           torch.from_numpy(ks2).to(dev), torch.from_numpy(Ls2).to(dev), 10, plan)
    for a, b in zip(ref2, got2):
        assert (a == b).all()
    o2 = oracle.search(base, g, q[:m], ent2, 10, 24)
    assert (got2[0] == o2["ids"]).all()
    assert (got2[2][:, 2] == o2["hops"]).all()


def test_noalloc_search_rejects_a_batch_beyond_its_scratch():
    ann = _ann()
    dev = torch.device("cuda:0")
    one = torch.zeros((1, 4), dtype=torch.float32, device=dev)
    gi = torch.zeros((1, 1), dtype=torch.int32, device=dev)
    ki = torch.ones(1, dtype=torch.int32, device=dev)
    import ctypes
    st = ann._lib.ann_search_noalloc(ctypes.c_void_p(one.data_ptr()), 1, 4,
                                     ctypes.c_void_p(gi.data_ptr()), 1,
                                     ctypes.c_void_p(one.data_ptr()), ann.ANN_NOALLOC_MAX_QUERIES + 1,
                                     None, 0, ctypes.c_void_p(ki.data_ptr()),
                                     ctypes.c_void_p(ki.data_ptr()), 1,
                                     ctypes.c_void_p(gi.data_ptr()), ctypes.c_void_p(one.data_ptr()),
                                     None, None, 0, None, None)
    assert st == ann.ANN_EINVAL and "at most" in ann.last_error()
