"""GPU parity at the serving workload's size (10M x 128 integers, R = 64 from
the all-pairs 128-NN): sampled graph rows, the medoid and reachability
against the oracle; the learned entry over 1,024 hubs for all 10,000 queries;
and a served mix of requests (k 10 and 100, 30 % of the queries
out-of-distribution, medoid fallback at a tuned threshold) whose rows are
checked against the oracle's search from the same entries."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_15986_amd import synth
from tests.common import say

pytestmark = pytest.mark.gpu


def _ann():
    from paper_2506_15986_amd import ann
    return ann


@pytest.fixture(scope="module")
def big():
    ann = _ann()
    from paper_2506_15986_amd import gate
    w = synth.WORKLOADS["sift10m"]
    say("case: sift10m data (10M x 128)")
    base = synth.base(w)
    q = synth.queries(w)
    dev = torch.device("cuda:0")
    bd, qd = torch.from_numpy(base).to(dev), torch.from_numpy(q).to(dev)
    say("case: sift10m graph build (all-pairs 128-NN, R 64)")
    index = gate.build_index(bd, 128, 64, 1.2)
    return dict(w=w, base=base, q=q, bd=bd, qd=qd, index=index, ann=ann,
                graph=index.graph.cpu().numpy())


def test_10m_graph_rows_medoid_and_reachability(big):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order
    base, g, index = big["base"], big["graph"], big["index"]
    n, R = g.shape
    say("case: medoid at 10M")
    assert index.medoid == oracle.medoid(base)
    say("case: sampled rows: exact 128-NN then alpha 1.2 pruning")
    rows = np.random.default_rng(41).choice(n, 8, replace=False)
    ids, d2 = oracle.knn(base, base[rows], 129)
    for r, p in enumerate(rows):
        keep = ids[r] != p
        cid, cd2 = ids[r][keep][:128], d2[r][keep][:128]
        sub = np.concatenate([base[p:p + 1], base[cid]])
        cand = np.full((sub.shape[0], 128), -1, np.int32)
        cand[0] = np.arange(1, 129, dtype=np.int32)
        dd = np.zeros((sub.shape[0], 128))
        dd[0] = cd2
        pr = oracle.alpha_prune(sub, cand, dd, R, 1.2)[0]
        want = np.where(pr >= 0, cid[np.maximum(pr - 1, 0)], -1)
        assert (g[p, :R - 2] == want[:R - 2]).all(), p
    say("case: every node reachable from the medoid and reaching it")
    assert ((g >= -1) & (g < n)).all()
    idx = np.where(g >= 0, g, np.arange(n, dtype=np.int32)[:, None]).reshape(-1)   # -1 -> self
    A = sp.csr_matrix((np.ones(idx.size, np.int8), idx, np.arange(n + 1, dtype=np.int64) * R),
                      shape=(n, n))
    del idx
    assert breadth_first_order(A, index.medoid, directed=True,
                               return_predecessors=False).shape[0] == n
    At = A.T.tocsr()
    del A
    assert breadth_first_order(At, index.medoid, directed=True,
                               return_predecessors=False).shape[0] == n


def test_10m_gate_entries_and_served_mix(big):
    import dataclasses

    from tests.common import near_tie_certificate
    ann = big["ann"]
    from paper_2506_15986_amd import gate, serve
    base, q, bd, qd, index, g = (big[x] for x in ("base", "q", "bd", "qd", "index", "graph"))
    nq = q.shape[0]
    w = synth.scaled(big["w"], n_train=30_000)
    say("case: GATE build at 10M (1024 hubs, 30,000 training queries)")
    tq = torch.from_numpy(synth.train_queries(w)).to(bd.device)
    gm = gate.build_gate(index, tq, w, log=say)
    L_h = int(gm.model.c.L_h)
    say("case: entry selection for all %d queries at L_h = %d" % (nq, L_h))
    ent, _, bh = ann.ann_entry_select(gm.model, qd, want_score=True)
    qe_d = gm.qtower.forward(qd)
    torch.cuda.synchronize()
    ent_h, bh_h, qe = ent.cpu().numpy(), bh.cpu().numpy(), qe_d.cpu().numpy()
    he, hg = gm.hub_emb.cpu().numpy(), gm.hub_graph.cpu().numpy()
    hub_ids = gm.hub_ids.cpu().numpy()
    _, _, ref_bh = oracle.entry_select(qe, he, hg, hub_ids, L_h, -np.inf, index.medoid,
                                       gm.hub_entry)
    assert (ent_h == hub_ids[bh_h]).all()
    mis = np.flatnonzero(bh_h != ref_bh)
    say("entry selection: %d of %d best hubs differ from the oracle's" % (mis.size, nq))
    if mis.size:
        md = torch.from_numpy(mis).to(bd.device)
        from tests.common import hub_search_traced
        tids, ttr = hub_search_traced(ann, gm, qe_d[md].contiguous(), L_h)
        assert (tids == bh_h[mis]).all()
        rt = oracle.search(he, hg, qe[mis], gm.hub_entry, 1, L_h, trace_cap=1024)
        for t in range(mis.size):
            assert near_tie_certificate(he, hg, qe[mis[t]], gm.hub_entry, L_h, ttr[t],
                                        rt["trace"][t]), mis[t]
    assert mis.size <= nq // 100
    say("case: medoid fallback threshold on training queries of the mix")
    wm = dataclasses.replace(w, shift=0.3, shifted_frac=0.3)
    tm = tq[:5000].contiguous()
    theta, rows = gate.tune_theta(index, gm, tm, ann.ann_gt_knn(bd, tm, 10)[0], 320)
    say("theta %s, sweep %s" % (theta, rows))
    del tq, tm
    say("case: a served mix (k 10 at L 320, k 100 at L 640)")
    qm = synth.queries(wm, 4000)
    plan = ann.default_plan(base.shape[0], base.shape[1], g.shape[1], 640)
    srv = serve.Server(bd, index.graph, index.medoid, model=gm.model, slots=4, slot_rows=1024,
                       k_max=100, L_max=640, plan=plan)
    sched = serve.poisson_schedule(qm, 1e12, sizes=(1, 300), kL=((10, 320), (100, 640)), seed=5)
    st = srv.serve(sched)
    say("served: %s" % st)
    assert st["requests"] == len(sched) and st["max_slots_busy"] >= 2
    # sampled rows against the oracle from the same entries (FP32 exact on integers)
    r = np.random.default_rng(42)
    picks = []
    for req in sched:
        for row in r.choice(req.queries.shape[0], min(2, req.queries.shape[0]), replace=False):
            picks.append((req, int(row)))
    picks = [picks[i] for i in r.choice(len(picks), 48, replace=False)]
    for kq, Lq in ((10, 320), (100, 640)):
        sel = [(req, row) for req, row in picks if req.k == kq]
        if not sel:
            continue
        qs = np.stack([req.queries[row] for req, row in sel])
        es = ann.ann_entry_select(gm.model, torch.from_numpy(qs).to(bd.device))[0].cpu().numpy()
        ref = oracle.search(base, g, qs, es, kq, Lq)
        got = np.stack([req.ids[row] for req, row in sel])
        assert (got == ref["ids"]).all(), kq
        gd = np.stack([req.dist[row] for req, row in sel]).astype(np.float64)
        assert (gd == ref["d2"]).all(), kq
    gm.model.c.theta = -np.inf
