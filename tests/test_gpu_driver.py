"""GPU tests of the batch driver: the autotuner, one-call query batches and
their HIP graphs (C-ABI), against the separate entry points and the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_15986_amd import synth
from tests.common import int_index, say, tiny_index

pytestmark = pytest.mark.gpu


def _ann():
    from paper_2506_15986_amd import ann
    return ann


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _model(ix, nh=64, L_h=16):
    """An entry model on the tiny index with untrained towers (the driver's
    results do not depend on what the towers learned)."""
    ann = _ann()
    base, w = ix["base"], ix["w"]
    d = base.shape[1]
    init = synth.kmeans_init(w, base.shape[0], nh)
    hub_ids = np.sort(init).astype(np.int32)
    qp = synth.tower_init(w, [(64, d), (32, 64)])
    hp = synth.tower_init(w, [(64, d), (32, 64)])
    qt, ht = ann.Tower(*qp), ann.Tower(*hp)
    hemb = ht.forward(_dev(base[hub_ids]))
    hg, hub_entry = ann.ann_navgraph_build(hemb, 8)
    torch.cuda.synchronize()
    return ann.EntryModel(qt, hemb, hg, _dev(hub_ids), hub_entry, ix["medoid"], L_h=L_h)


def test_autotune_returns_a_candidate_with_identical_results():
    ann = _ann()
    ix = int_index()
    n, d = ix["base"].shape
    R = ix["graph"].shape[1]
    nq, L = ix["q"].shape[0], 64
    say("case: autotune L=%d nq=%d" % (L, nq))
    base, g, q = _dev(ix["base"]), _dev(ix["graph"]), _dev(ix["q"])
    best, times = ann.ann_autotune_search(base, g, q, None, ix["medoid"], 10, L, 10, L, reps=2)
    torch.cuda.synchronize()
    cands = [p.as_dict() for p, _ in times]
    assert best.as_dict() in cands
    assert all(ms > 0 for _, ms in times)
    assert min(ms for _, ms in times) == dict((tuple(p.as_dict().items()), ms)
                                              for p, ms in times)[tuple(best.as_dict().items())]
    say("case: autotuned plan vs oracle")
    ids, dist, st, _ = ann.ann_search(base, g, q, None, ix["medoid"], 10, L, k_max=10, plan=best)
    torch.cuda.synchronize()
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L)
    assert (ids.cpu().numpy() == ref["ids"]).all()
    assert (st.cpu().numpy()[:, 2] == ref["hops"]).all()


def test_query_run_equals_separate_calls():
    ann = _ann()
    ix = tiny_index()
    model = _model(ix)
    base, g, q = _dev(ix["base"]), _dev(ix["graph"]), _dev(ix["q"])
    nq = q.shape[0]
    rng = np.random.default_rng(5)
    ks = _dev(rng.integers(1, 11, nq).astype(np.int32))
    Ls = _dev(rng.integers(10, 65, nq).astype(np.int32))
    say("case: query_run ALL vs entry_select + search")
    b = ann.QueryBatch(base, g, ix["medoid"], q, ks, Ls, 10, model=model)
    ids, dist, st = b.run()
    ent, _, _ = ann.ann_entry_select(model, q)
    ids2, dist2, st2, _ = ann.ann_search(base, g, q, ent, ix["medoid"], ks, Ls, k_max=10,
                                         plan=b.plan)
    torch.cuda.synchronize()
    assert (b.entry_ids.cpu().numpy() == ent.cpu().numpy()).all()
    assert (ids.cpu().numpy() == ids2.cpu().numpy()).all()
    assert (dist.cpu().numpy().view(np.uint32) == dist2.cpu().numpy().view(np.uint32)).all()
    assert (st.cpu().numpy() == st2.cpu().numpy()).all()


def test_query_graph_replays_match_eager():
    ann = _ann()
    ix = tiny_index()
    model = _model(ix)
    base, g = _dev(ix["base"]), _dev(ix["graph"])
    q = _dev(ix["q"])
    nq = q.shape[0]
    b = ann.QueryBatch(base, g, ix["medoid"], q, 10, 32, 10, model=model)
    say("case: eager reference")
    ids_e, dist_e, _ = [t.clone() for t in b.run()]
    torch.cuda.synchronize()
    ref_ids, ref_dist = ids_e.cpu().numpy(), dist_e.cpu().numpy()
    say("case: graph create")
    gx = b.graph_exec(ann.ANN_STAGE_ALL)
    for r in range(3):
        say("case: replay %d" % r)
        b.ids.fill_(-7)
        b.dist.zero_()
        b.entry_ids.fill_(-1)
        torch.cuda.synchronize()
        gx.launch()
        torch.cuda.synchronize()
        assert (b.ids.cpu().numpy() == ref_ids).all(), r
        assert (b.dist.cpu().numpy().view(np.uint32) == ref_dist.view(np.uint32)).all(), r
        # eager work between replays
        ann.ann_search(base, g, q, None, ix["medoid"], 10, 16, k_max=10)
        torch.cuda.synchronize()
    say("case: replay on new query contents")
    q2 = np.ascontiguousarray(ix["q"][::-1])
    q.copy_(_dev(q2))
    torch.cuda.synchronize()
    gx.launch()
    torch.cuda.synchronize()
    ent, _, _ = ann.ann_entry_select(model, _dev(q2))
    ids2, _, _, _ = ann.ann_search(base, g, _dev(q2), ent, ix["medoid"], 10, 32, k_max=10,
                                   plan=b.plan)
    torch.cuda.synchronize()
    assert (b.ids.cpu().numpy() == ids2.cpu().numpy()).all()
    assert (b.ids.cpu().numpy() == ref_ids[::-1]).all()
    gx.close()


def test_search_only_graph_from_the_medoid_matches_oracle():
    ann = _ann()
    ix = int_index()
    base, g, q = _dev(ix["base"]), _dev(ix["graph"]), _dev(ix["q"])
    say("case: search-only graph, medoid entry")
    b = ann.QueryBatch(base, g, ix["medoid"], q, 10, 48, 10)
    gx = b.graph_exec(ann.ANN_STAGE_SEARCH)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, 48)
    for r in range(2):
        b.ids.fill_(-7)
        torch.cuda.synchronize()
        gx.launch()
        torch.cuda.synchronize()
        assert (b.ids.cpu().numpy() == ref["ids"]).all(), r
    gx.close()


def test_batches_side_by_side_on_streams_with_their_own_queues():
    # two batches' graphs replayed at once on ann_stream_create streams, with
    # capped persistent grids so that both launches are resident together;
    # each batch's rows equal the oracle's
    ann = _ann()
    ix = int_index()
    base, g, q = _dev(ix["base"]), _dev(ix["graph"]), _dev(ix["q"])
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, 48)
    plan = ann.default_plan(base.shape[0], base.shape[1], g.shape[1], 48)
    plan = ann.make_plan(**dict(plan.as_dict(), waves_per_block=4, blocks=64,
                                waves_per_query=1))
    say("case: two dedicated streams, plan %s" % plan)
    streams = [ann.ann_stream_create() for _ in range(2)]
    batches = [ann.QueryBatch(base, g, ix["medoid"], q, 10, 48, 10, plan=plan) for _ in range(2)]
    graphs = [bx.graph_exec(ann.ANN_STAGE_SEARCH) for bx in batches]
    for r in range(3):
        for bx in batches:
            bx.ids.fill_(-7)
        torch.cuda.synchronize()
        for gx, st in zip(graphs, streams):
            gx.launch(stream=st)
        torch.cuda.synchronize()
        for bx in batches:
            assert (bx.ids.cpu().numpy() == ref["ids"]).all(), r
    for gx in graphs:
        gx.close()
    for st in streams:
        ann.ann_stream_destroy(st)
    torch.cuda.synchronize()
    say("case: the process-wide dedicated streams")
    assert ann.dedicated_stream(0).cuda_stream == ann.dedicated_stream(0).cuda_stream
    assert ann.dedicated_stream(0).cuda_stream != ann.dedicated_stream(1).cuda_stream


def test_autotune_on_float_data_and_a_tuned_hub_plan():
    # grid data: FP32 distances are not exact, so plans of different gather
    # groups may order near-ties differently; each group checks against its own
    ann = _ann()
    ix = tiny_index()
    base, g, q = _dev(ix["base"]), _dev(ix["graph"]), _dev(ix["q"])
    say("case: autotune on float data")
    best, times = ann.ann_autotune_search(base, g, q, None, ix["medoid"], 10, 32, 10, 32, reps=1)
    torch.cuda.synchronize()
    assert {p.group for p, _ in times} == {4, 8, 16}     # d = 32: every group
    ids, dist, _, _ = ann.ann_search(base, g, q, None, ix["medoid"], 10, 32, k_max=10, plan=best)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, 32)
    d, rd = dist.cpu().numpy().astype(np.float64), ref["d2"]
    assert np.abs(d - rd).max() <= 1e-5 * max(rd.max(), 1e-6)
    assert (ids.cpu().numpy() == ref["ids"]).mean() >= 0.99
    say("case: tuned hub-search plan")
    model = _model(ix, L_h=24)
    e0, _, b0 = ann.ann_entry_select(model, q, want_score=True)
    plan = model.tune_hub_plan(q, reps=1)
    assert plan.pool_cap >= 24
    e1, _, b1 = ann.ann_entry_select(model, q, want_score=True)
    torch.cuda.synchronize()
    qe = model.qtower.forward(q).cpu().numpy().astype(np.float64)
    he = model.hub_emb.cpu().numpy().astype(np.float64)
    cos = qe @ he.T
    b0, b1 = b0.cpu().numpy(), b1.cpu().numpy()
    rows = np.arange(len(b0))
    assert (np.abs(cos[rows, b0] - cos[rows, b1]) <= 1e-5).all()
    assert (b0 == b1).mean() >= 0.98


def test_tune_hub_search_width():
    # the chosen width's best hubs match the exact cosine argmax on the sample
    ann = _ann()
    ix = tiny_index()
    model = _model(ix, L_h=32)
    q = _dev(ix["q"])
    say("case: hub-search width tuning")
    L = model.tune_L_h(q, agree=0.99, ladder=(4, 8, 16, 32, 64))
    assert L in (4, 8, 16, 32, 64) and model.c.L_h == L
    rates = dict(model.L_h_rates)
    assert rates[L] >= 0.99 or L == 64
    assert all(r < 0.99 for l, r in rates.items() if l < L)
    _, _, bh = ann.ann_entry_select(model, q, want_score=True)
    qe = model.qtower.forward(q).cpu().numpy().astype(np.float64)
    cos = qe @ model.hub_emb.cpu().numpy().astype(np.float64).T
    hit = np.abs(cos[np.arange(len(qe)), bh.cpu().numpy()] - cos.max(1)) <= 1e-6
    assert hit.mean() >= 0.99 or L == 64


def test_training_keeps_the_epoch_with_the_best_held_out_agreement():
    # select_best: the towers left after training are the ones of the best
    # epoch on the held-out queries (recomputed here from the returned towers)
    from paper_2506_15986_amd import gate
    ann = _ann()
    w = synth.scaled(synth.WORKLOADS["tiny"], n=10_000, n_queries=100, n_train=4_000)
    base = _dev(synth.base(w))
    say("case: epoch selection on the tiny workload")
    index = gate.build_index(base, 64, 16, 1.2, w=w, log=None)
    tq = _dev(synth.train_queries(w))
    gd = gate.prepare_gate(index, tq, w, n_hubs=64, log=lambda *a: None)
    g = gate.train_gate(index, gd, tq, w, hidden=32, dout=16, epochs=6, batch=256,
                        select_best=True, tune_L_h=False, log=lambda *a: None)
    curve = g.info["val_curve"]
    assert [e for e, _ in curve] == list(range(1, 7))
    best = max(a for _, a in curve)
    assert g.info["selected_epoch"] == next(e for e, a in curve if a == best)
    nt = tq.shape[0] - int(round(0.1 * tq.shape[0]))
    hemb = g.htower.forward(g.hub_in)
    hg, he = ann.ann_navgraph_build(hemb, 16)
    mdl = ann.EntryModel(g.qtower, hemb, hg, gd.hub_ids, he, index.medoid, L_h=32)
    _, _, bh = ann.ann_entry_select(mdl, tq[nt:].contiguous(), want_score=True)
    acc = float((bh == gd.labels[nt:]).float().mean().item())
    assert round(acc, 4) == best
