"""GPU parity of the learned entry model: tower forward, training gradients
(against the oracle's float64 two-tower model on the same BF16 operands),
Adam, the hub navigation graph, entry selection and training labels."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import towers as T
from paper_2506_15986_amd import synth
from tests.common import int_index, say, tiny_index, tower_certificate

pytestmark = pytest.mark.gpu


def _ann():
    from paper_2506_15986_amd import ann
    return ann


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _setup(nh=64, hidden=128, dout=64):
    ix = tiny_index()
    base, w = ix["base"], ix["w"]
    d = base.shape[1]
    init = synth.kmeans_init(w, base.shape[0], nh)
    km = oracle.kmeans_hubs(base, nh, 20, init)
    feat, _ = oracle.hub_features(base, ix["graph"], ix["medoid"], km["hub_ids"], km["assign"],
                                  km["centroids"])
    hub_in = np.concatenate([base[km["hub_ids"]], feat.astype(np.float32)], axis=1)
    qp = synth.tower_init(w, [(hidden, d), (dout, hidden)])
    hp = synth.tower_init(w, [(hidden, d + 32), (dout, hidden)])
    return ix, km, hub_in, qp, hp


def test_tower_forward_matches_oracle():
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    say("case: tower forward")
    for params, x in ((qp, ix["q"]), (hp, hub_in)):
        t = ann.Tower(*params)
        e = t.forward(_dev(x)).cpu().numpy()
        beyond, cert, unc = tower_certificate(params, x.astype(np.float64), e)
        say("tower rows beyond 1e-4: %d, certified by BF16 re-rounding of a hidden element: %d"
            % (beyond, cert))
        assert not unc, unc
        assert np.allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-5)
    # a larger batch of queries (the 1M x 128 recipe's integers, scaled into
    # [-1, 1] as the entry model does)
    xi = int_index()["q"].astype(np.float64)
    qpi = synth.tower_init(ix["w"], [(128, 128), (64, 128)])
    t = ann.Tower(*qpi, in_scale=1.0 / 256)
    e = t.forward(_dev(xi.astype(np.float32))).cpu().numpy()
    beyond, cert, unc = tower_certificate(qpi, xi, e, in_scale=1.0 / 256)
    say("integer queries: rows beyond 1e-4: %d, certified: %d" % (beyond, cert))
    assert not unc, unc


def test_fused_tower_forward_equals_generic_forward():
    # inference runs both layers and the normalisation in one kernel when the
    # input rows are 16-byte aligned; a row pointer 4 bytes off takes the
    # generic path (input rounding, two GEMMs, normalisation).  The two must
    # give the same bits: same roundings, same MFMA step order, same sums.
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    xi = int_index()["q"].astype(np.float32)
    qpi = synth.tower_init(ix["w"], [(128, 128), (64, 128)])
    hp256 = synth.tower_init(ix["w"], [(256, hub_in.shape[1]), (128, 256)])
    for name, params, x, scale in (("query 32-128-64", qp, ix["q"], 1.0),
                                   ("hub 64-128-64", hp, hub_in, 1.0),
                                   ("query 128-128-64, scaled", qpi, xi, 1.0 / 256),
                                   ("hub 64-256-128", hp256, hub_in, 1.0)):
        say("case: fused against generic tower forward, %s" % name)
        t = ann.Tower(*params, in_scale=scale)
        xa = _dev(np.ascontiguousarray(x, dtype=np.float32))
        buf = torch.empty(xa.numel() + 1, dtype=torch.float32, device=xa.device)
        xm = buf[1:].view(xa.shape)
        xm.copy_(xa)
        assert xa.data_ptr() % 16 == 0 and xm.data_ptr() % 16 == 4
        ea, em = t.forward(xa), t.forward(xm)
        torch.cuda.synchronize()
        assert torch.equal(ea.view(torch.int32), em.view(torch.int32)), name


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("scale", [1.0, 0.0625])
def test_train_step_gradients_match_oracle(scale):
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    tq = synth.train_queries(ix["w"], 512)
    r = np.random.default_rng(1)
    labels = r.integers(0, hub_in.shape[0], size=tq.shape[0]).astype(np.int32)
    idx = r.permutation(tq.shape[0])[:256].astype(np.int32)
    say("case: train step gradients, input scale %g" % scale)
    qt, ht = ann.Tower(*qp, in_scale=scale), ann.Tower(*hp)
    loss, qe, he = ann.ann_train_step(qt, ht, _dev(tq), _dev(idx), _dev(labels), _dev(hub_in), 0.07,
                                      1e-3, 0, want_emb=True)
    torch.cuda.synchronize()
    ref_loss, gq, gh, eq, eh = T.train_step_grads(qp, hp, tq[idx].astype(np.float64),
                                                  hub_in.astype(np.float64), labels[idx], 0.07,
                                                  bf16=True, q_scale=scale)
    assert abs(loss.item() - ref_loss) <= 1e-4 * abs(ref_loss)
    for got, ref in zip([t.cpu().numpy() for t in qt.g + ht.g], list(gq) + list(gh)):
        assert _rel(got, ref) <= 1e-3
    # a second identical step gives identical bits (fixed-order reductions)
    g1 = [t.clone() for t in qt.g + ht.g]
    ann.ann_train_step(qt, ht, _dev(tq), _dev(idx), _dev(labels), _dev(hub_in), 0.07, 1e-3, 0)
    torch.cuda.synchronize()
    for a, b in zip(g1, qt.g + ht.g):
        assert torch.equal(a, b)


def test_adam_step_matches_oracle_update():
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    tq = synth.train_queries(ix["w"], 256)
    labels = np.arange(256, dtype=np.int32) % hub_in.shape[0]
    idx = np.arange(256, dtype=np.int32)
    say("case: adam")
    qt, ht = ann.Tower(*qp), ann.Tower(*hp)
    ann.ann_train_step(qt, ht, _dev(tq), _dev(idx), _dev(labels), _dev(hub_in), 0.07, 1e-3, 0)
    grads = [t.cpu().numpy().astype(np.float64) for t in qt.g]
    ann.ann_train_step(qt, ht, _dev(tq), _dev(idx), _dev(labels), _dev(hub_in), 0.07, 1e-3, 1)
    torch.cuda.synchronize()
    for p0, g, p1 in zip(qp, grads, [t.cpu().numpy() for t in qt.params()]):
        want, _, _ = T.adam_update(np.asarray(p0, np.float64), g, 0 * g, 0 * g, 1, 1e-3)
        assert np.allclose(p1, want, rtol=1e-6, atol=1e-7)
    # BF16 copies follow the masters
    w1b = qt.W1b.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(w1b.view(np.float32),
                          T.bf16_round(qt.W1.cpu().numpy().astype(np.float64)).astype(np.float32))


def test_training_reduces_loss():
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    tq = synth.train_queries(ix["w"], 1000)
    # label = nearest hub by L2 (a learnable target)
    lab, _ = oracle.knn(ix["base"][km["hub_ids"]], tq, 1)
    labels = lab[:, 0].astype(np.int32)
    qt, ht = ann.Tower(*qp), ann.Tower(*hp)
    tq_d, lab_d, hub_d = _dev(tq), _dev(labels), _dev(hub_in)
    say("case: training reduces loss")
    losses = []
    for step in range(1, 61):
        idx = _dev(synth.batch_order(ix["w"], 1000, step)[:256].astype(np.int32))
        loss, _, _ = ann.ann_train_step(qt, ht, tq_d, idx, lab_d, hub_d, 0.07, 3e-3, step)
        losses.append(loss.item())
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:5])


@pytest.mark.skip(reason="went silent on the GPU (killed after 180 s) in its first run with the "
                         "first navgraph / hub-search kernels; no cause was found by reading, by CPU "
                         "emulation of the search or in the assembly, so those kernels were taken "
                         "out and this case is kept off the GPU")
def test_navgraph_and_entry_select_match_oracle():
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    say("case: navgraph + entry select")
    qt, ht = ann.Tower(*qp), ann.Tower(*hp)
    hemb = ht.forward(_dev(hub_in))
    hg, hub_entry = ann.ann_navgraph_build(hemb, 16)
    torch.cuda.synchronize()
    he = hemb.cpu().numpy()
    assert (hg.cpu().numpy() == oracle.hub_graph(he, 16)).all()
    assert hub_entry == oracle.hub_medoid(he)
    hub_ids = _dev(km["hub_ids"])
    for Lh in (8, 32, 64):
        model = ann.EntryModel(qt, hemb, hg, hub_ids, hub_entry, ix["medoid"], L_h=Lh)
        ent, sc, bh = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True)
        qe = qt.forward(_dev(ix["q"])).cpu().numpy()
        torch.cuda.synchronize()
        ref_ent, ref_sc, ref_bh = oracle.entry_select(qe, he, hg.cpu().numpy(), km["hub_ids"], Lh,
                                                      -math.inf, ix["medoid"], hub_entry)
        got_bh = bh.cpu().numpy()
        cos = qe.astype(np.float64) @ he.astype(np.float64).T
        for i in range(len(got_bh)):
            if got_bh[i] != ref_bh[i]:
                # only a near tie between the two choices may differ
                assert abs(cos[i, got_bh[i]] - cos[i, ref_bh[i]]) <= 1e-5
        assert (got_bh == ref_bh).mean() >= 0.98
        assert np.allclose(sc.cpu().numpy(), ref_sc, atol=1e-5)
        if Lh >= 64:
            assert (got_bh == np.argmax(cos, axis=1)).mean() >= 0.98
    # theta above every cosine -> medoid everywhere
    model = ann.EntryModel(qt, hemb, hg, hub_ids, hub_entry, ix["medoid"], L_h=16, theta=2.0)
    ent, _, _ = ann.ann_entry_select(model, _dev(ix["q"]))
    assert (ent.cpu().numpy() == ix["medoid"]).all()


def test_hub_graph_and_entry_select_via_search_engines():
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    say("case: hub embeddings")
    qt, ht = ann.Tower(*qp), ann.Tower(*hp)
    hemb = ht.forward(_dev(hub_in))
    torch.cuda.synchronize()
    he = hemb.cpu().numpy()
    say("case: navigation graph")
    hg, hub_entry = ann.ann_navgraph_build(hemb, 16)
    torch.cuda.synchronize()
    ref_hg = oracle.hub_graph(he, 16)
    got_hg = hg.cpu().numpy()
    d2 = ((he[:, None, :].astype(np.float64) - he[None, :, :]) ** 2).sum(-1)
    for i in range(he.shape[0]):
        for t in range(16):
            if got_hg[i, t] != ref_hg[i, t]:   # only FP64 near-ties may swap
                assert abs(d2[i, got_hg[i, t]] - d2[i, ref_hg[i, t]]) <= 1e-12
    assert (got_hg == ref_hg).mean() >= 0.99
    assert hub_entry == oracle.hub_medoid(he)
    hub_ids = _dev(km["hub_ids"])
    qe = qt.forward(_dev(ix["q"])).cpu().numpy()
    cos = qe.astype(np.float64) @ he.astype(np.float64).T
    for Lh in (8, 32, 64):
        say("case: entry select L_h=%d" % Lh)
        model = ann.EntryModel(qt, hemb, hg, hub_ids, hub_entry, ix["medoid"], L_h=Lh)
        ent, sc, bh = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True)
        torch.cuda.synchronize()
        ref_ent, ref_sc, ref_bh = oracle.entry_select(qe, he, ref_hg, km["hub_ids"], Lh,
                                                      -math.inf, ix["medoid"], hub_entry)
        got_bh = bh.cpu().numpy()
        for i in range(len(got_bh)):
            if got_bh[i] != ref_bh[i]:   # FP32 search vs FP64 oracle: near ties only
                assert abs(cos[i, got_bh[i]] - cos[i, ref_bh[i]]) <= 1e-5
        assert (got_bh == ref_bh).mean() >= 0.98
        assert (ent.cpu().numpy() == km["hub_ids"][got_bh]).all()
        assert np.allclose(sc.cpu().numpy(), cos[np.arange(len(got_bh)), got_bh], atol=1e-5)
        if Lh >= 64:
            assert (got_bh == np.argmax(cos, axis=1)).mean() >= 0.98
    say("case: entry select theta fallback")
    model = ann.EntryModel(qt, hemb, hg, hub_ids, hub_entry, ix["medoid"], L_h=16, theta=2.0)
    ent, _, _ = ann.ann_entry_select(model, _dev(ix["q"]))
    torch.cuda.synchronize()
    assert (ent.cpu().numpy() == ix["medoid"]).all()
    # theta in a gap of the scores near their median: the queries below it
    # fall back to the medoid, the others keep their hub, as in the oracle
    model = ann.EntryModel(qt, hemb, hg, hub_ids, hub_entry, ix["medoid"], L_h=16)
    _, sc, bh = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True)
    sc, bh = sc.cpu().numpy().astype(np.float64), bh.cpu().numpy()
    srt = np.sort(sc)
    gaps = [t for t in range(len(srt) // 4, 3 * len(srt) // 4) if srt[t + 1] - srt[t] > 2e-5]
    t = gaps[len(gaps) // 2]
    theta = 0.5 * (srt[t] + srt[t + 1])
    say("case: partial fallback, theta %.6f (%d of %d below)" % (theta, t + 1, len(sc)))
    model = ann.EntryModel(qt, hemb, hg, hub_ids, hub_entry, ix["medoid"], L_h=16, theta=theta)
    ent, sc2, bh2 = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True)
    torch.cuda.synchronize()
    ent, bh2 = ent.cpu().numpy(), bh2.cpu().numpy()
    assert (bh2 == bh).all()
    below = sc < theta
    assert below.sum() == t + 1
    assert (ent[below] == ix["medoid"]).all()
    assert (ent[~below] == km["hub_ids"][bh[~below]]).all()
    # the same model behind a library handle gives the same rows, bit for bit
    say("case: entry select through a model handle")
    h = ann.ann_entry_model_create(model)
    try:
        ent3, sc3, bh3 = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True, handle=h)
        torch.cuda.synchronize()
    finally:
        ann.ann_entry_model_destroy(h)
    assert (ent3.cpu().numpy() == ent).all() and (bh3.cpu().numpy() == bh2).all()
    assert (sc3.cpu().numpy().view(np.uint32) == sc2.cpu().numpy().view(np.uint32)).all()
    ref_ent, ref_sc, ref_bh = oracle.entry_select(qe, he, ref_hg, km["hub_ids"], 16, theta,
                                                  ix["medoid"], hub_entry)
    same = ref_bh == bh
    assert same.mean() >= 0.98
    assert (ref_ent[same] == ent[same]).all()


@pytest.mark.skip(reason="its label-mode search kernel went silent on the GPU (killed after 180 s) "
                         "twice, the second time after a fix for duplicated kernel symbols; the "
                         "label-mode kernel was switched off and labels now come from the plain "
                         "search kernel (test_ladder_labels_match_oracle); the old call signature "
                         "no longer exists, so this case cannot run")
@pytest.mark.parametrize("which", ["tiny", "int"])
def test_labels_match_oracle(which):
    ix = tiny_index() if which == "tiny" else int_index()
    base, g, w = ix["base"], ix["graph"], ix["w"]
    nh, M, L = 64, 8, 64
    init = synth.kmeans_init(w, base.shape[0], nh)
    km = oracle.kmeans_hubs(base, nh, 20, init)
    tq = synth.train_queries(w, 300)
    truth, _ = oracle.knn(base, tq, 10)
    cand, _ = oracle.knn(base[km["hub_ids"]], tq, M)
    say("case: labels %s" % which)
    ref_lab, ref_tab = oracle.make_labels(base, g, tq, truth, cand, km["hub_ids"], L, 10)
    lab, tab, flags = _ann().ann_make_labels(_dev(base), _dev(g), _dev(tq), _dev(truth), 10,
                                             _dev(cand), _dev(km["hub_ids"]), L)
    torch.cuda.synchronize()
    lab, tab, flags = lab.cpu().numpy(), tab.cpu().numpy(), flags.cpu().numpy()
    assert (flags == 0).all()
    assert (lab == ref_lab).all()
    hit = tab >= 0
    assert (tab[hit] == ref_tab[hit]).all()
    assert (ref_tab[tab == -1] == -1).all()
    for i, m in zip(*np.where(tab == -2)):
        best = min(v for v in tab[i] if v >= 0)
        assert ref_tab[i, m] == -1 or ref_tab[i, m] > best


@pytest.mark.parametrize("which", ["tiny", "int"])
def test_ladder_labels_match_oracle(which):
    ix = tiny_index() if which == "tiny" else int_index()
    base, g, w = ix["base"], ix["graph"], ix["w"]
    nh, M, ladder = 64, 6, [10, 16, 32, 64]
    init = synth.kmeans_init(w, base.shape[0], nh)
    km = oracle.kmeans_hubs(base, nh, 20, init)
    tq = synth.train_queries(w, 200)
    truth, _ = oracle.knn(base, tq, 10)
    cand, _ = oracle.knn(base[km["hub_ids"]], tq, M)
    say("case: ladder labels %s (oracle)" % which)
    ref_lab, ref_tab = oracle.make_labels(base, g, tq, truth, cand, km["hub_ids"], ladder, 10)
    say("case: ladder labels %s (gpu)" % which)
    lab, tab, flags = _ann().ann_make_labels(_dev(base), _dev(g), _dev(tq), _dev(truth), 10,
                                             _dev(cand), _dev(km["hub_ids"]), ladder)
    torch.cuda.synchronize()
    say("case: ladder labels %s (compare)" % which)
    lab, tab, flags = lab.cpu().numpy(), tab.cpu().numpy(), flags.cpu().numpy()
    assert (flags == 0).all()
    if which == "int":      # FP32 distances are exact: identical trajectories
        assert (tab == ref_tab).all() and (lab == ref_lab).all()
        return
    # grid data: FP32 vs FP64 near ties may move a cost; every differing cost
    # needs a certificate, and labels may differ only where a cost does
    from tests.common import near_tie_certificate
    ann = _ann()
    bad = np.argwhere(tab != ref_tab)
    say("case: ladder labels tiny: %d of %d costs differ, certifying" % (len(bad), tab.size))
    assert len(bad) <= tab.size // 20
    plan = ann.default_plan(base.shape[0], base.shape[1], g.shape[1], max(ladder))
    plan.filter, plan.visited_log2 = ann.ANN_FILTER_ID32, 13
    for i, m in bad:
        hub = int(km["hub_ids"][cand[i, m]])
        certified = False
        for L in ladder:
            ids, dd, _, tr = ann.ann_search(_dev(base), _dev(g), _dev(tq[i:i + 1]),
                                            _dev(np.array([hub], np.int32)), 0, 10, L, plan=plan,
                                            trace_cap=1024)
            ids, dd, tr = ids.cpu().numpy()[0], dd.cpu().numpy()[0], tr.cpu().numpy()[0]
            ref = oracle.search(base, g, tq[i:i + 1], hub, 10, L, trace_cap=1024)
            if not (tr == ref["trace"][0]).all():
                # the trajectories part at a near tie (first differing expansion)
                certified = near_tie_certificate(base, g, tq[i], hub, L, tr, ref["trace"][0])
                break
            if set(ids.tolist()) != set(ref["ids"][0].tolist()):
                # the same trajectory, so the same visited set; the top 10 of
                # it differ only if its 10th and 11th distances are near tied
                seen = {hub}
                for pnode in tr[tr >= 0]:
                    seen.update(int(v) for v in g[pnode] if v >= 0)
                ds = sorted(oracle.sqdist(tq[i], base[v]) for v in seen)
                certified = len(ds) > 10 and abs(ds[9] - ds[10]) <= 1e-5 * max(ds[9], 1e-30)
                break
        assert certified, (int(i), int(m))
    diff_rows = set(int(i) for i, _ in bad)
    assert all(int(i) in diff_rows for i in np.flatnonzero(lab != ref_lab))


@pytest.mark.parametrize("P,N", [(4, 12), (1, 0), (8, 60)])
def test_hub_anchored_step_gradients_match_oracle(P, N):
    # Eq. 4 over per-hub queues: 16 hubs of the batch, P positives and N
    # negatives each (rows with repeats, as sampling with replacement gives)
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    tq = synth.train_queries(ix["w"], 512)
    r = np.random.default_rng(P * 100 + N)
    hubs = r.choice(hub_in.shape[0], 16, replace=False).astype(np.int32)
    q_idx = r.integers(0, tq.shape[0], size=16 * (P + N)).astype(np.int32)
    say("case: hub-anchored step, P=%d N=%d" % (P, N))
    qt, ht = ann.Tower(*qp, in_scale=0.0625), ann.Tower(*hp)
    loss, qe, he = ann.ann_train_step_hub(qt, ht, _dev(tq), _dev(q_idx), _dev(hubs), P, N,
                                          _dev(hub_in), 0.07, 1e-3, 0, want_emb=True)
    torch.cuda.synchronize()
    ref_loss, gq, gh, eq, eh = T.train_step_grads_hub(qp, hp, tq[q_idx].astype(np.float64),
                                                      hub_in[hubs].astype(np.float64), P, N, 0.07,
                                                      bf16=True, q_scale=0.0625)
    assert abs(loss.item() - ref_loss) <= 1e-4 * max(abs(ref_loss), 1.0)
    for got, ref in zip([t.cpu().numpy() for t in qt.g + ht.g], list(gq) + list(gh)):
        if np.linalg.norm(ref) == 0:
            assert np.abs(got).max() <= 1e-6
        else:
            assert _rel(got, ref) <= 1e-3


def test_hop_table_matches_oracle():
    # two batches of hubs (100 > 64); then a graph without its repair slots,
    # where some targets are unreachable (255)
    ann = _ann()
    ix = int_index()
    r = np.random.default_rng(5)
    hubs = r.choice(ix["base"].shape[0], 100, replace=False).astype(np.int32)
    targets = ix["truth"][:, 0].astype(np.int32)
    for name, g in (("graph", ix["graph"]), ("without repair slots", ix["graph"][:, :-2])):
        g = np.ascontiguousarray(g)
        say("case: hop table, %s" % name)
        H = ann.ann_hop_table(_dev(g), _dev(hubs), _dev(targets))
        torch.cuda.synchronize()
        ref = oracle.hop_table(g, hubs, targets)
        assert (H.cpu().numpy() == ref).all(), name
    assert (ref == 255).any()


def _queues_vs_oracle(ann, H, t_pos, t_neg):
    Hd = _dev(H)
    po, pq, no, nq_ = ann.ann_make_queues(Hd, t_pos, t_neg)
    torch.cuda.synchronize()
    po, pq, no, nq_ = (t.cpu().numpy() for t in (po, pq, no, nq_))
    pos, neg = oracle.sample_queues(H, t_pos, t_neg)
    assert po[0] == 0 and no[0] == 0
    assert (np.diff(po) == [len(x) for x in pos]).all()
    assert (np.diff(no) == [len(x) for x in neg]).all()
    for h in range(H.shape[1]):
        assert (pq[po[h]:po[h + 1]] == pos[h]).all(), h
        assert (nq_[no[h]:no[h + 1]] == neg[h]).all(), h
    return int(po[-1]), int(no[-1])


@pytest.mark.parametrize("t_pos,t_neg", [(3, 15), (0, 1), (1, 4), (200, 300)])
def test_definition4_queues_match_oracle(t_pos, t_neg):
    # the hop table of 100 hubs over 300 training queries' nearest neighbours,
    # on the graph without its repair slots (unreachable pairs present), then
    # a hand table: a hub that reaches no query, ragged tiles (nq = 300 is
    # not a multiple of 256) and hubs beyond the first 64
    ann = _ann()
    ix = int_index()
    g = np.ascontiguousarray(ix["graph"][:, :-2])
    r = np.random.default_rng(6)
    hubs = r.choice(ix["base"].shape[0], 100, replace=False).astype(np.int32)
    tq = synth.train_queries(ix["w"], 300)
    targets = oracle.knn(ix["base"], tq, 1)[0][:, 0].astype(np.int32)
    say("case: Definition 4 queues, t_pos %d, t_neg %d" % (t_pos, t_neg))
    H = ann.ann_hop_table(_dev(g), _dev(hubs), _dev(targets)).cpu().numpy()
    assert (H == 255).any()
    npos, nneg = _queues_vs_oracle(ann, H, t_pos, t_neg)
    assert npos > 0 and nneg > 0
    Hh = np.random.default_rng(7).integers(0, 40, size=(300, 70)).astype(np.uint8)
    Hh[:, 5] = 255                                    # reaches no query: no queues
    Hh[::3, 66] = 255
    Hh[17, 66] = 0
    _queues_vs_oracle(ann, Hh, t_pos, t_neg)


def test_fusion_tokens_match_their_definition():
    # p = x_hub * scale, U_s = (x_w - x_hub) * scale for the neighbour in slot s
    # (0 and mask 0 for an empty slot); FP32 subtract then an exact power-of-two
    # scale, so the result is bitwise that of the definition in FP32
    ann = _ann()
    ix = int_index()
    g = ix["graph"].copy()
    g[::5, -3:] = -1                                  # some empty slots
    hubs = np.array([0, 17, 19_999, 512, 17], np.int32)
    scale = 1.0 / 256
    say("case: fusion tokens")
    p, U, m = ann.ann_fusion_tokens(_dev(ix["base"]), _dev(g), _dev(hubs), scale)
    torch.cuda.synchronize()
    x = ix["base"]
    nb = g[hubs]
    want_m = (nb >= 0).astype(np.uint8)
    want_U = ((x[np.maximum(nb, 0)] - x[hubs][:, None, :]) * np.float32(scale)) * want_m[:, :, None]
    assert (m.cpu().numpy() == want_m).all()
    assert (p.cpu().numpy() == x[hubs] * np.float32(scale)).all()
    assert (U.cpu().numpy() == want_U.astype(np.float32)).all()


def test_fusion_forward_backward_match_oracle():
    # 4 heads of 16 channels over 32 tokens of 128 values; ragged masks and
    # one hub without tokens
    ann = _ann()
    r = np.random.default_rng(21)
    nh, S, d, heads, dk, df = 50, 32, 128, 4, 16, 64
    C = heads * dk
    Ws = [r.normal(0, 1 / np.sqrt(d), size=(C, d)), r.normal(0, 1 / np.sqrt(d), size=(C, d)),
          r.normal(0, 1 / np.sqrt(d), size=(C, d)), r.normal(0, 1 / np.sqrt(C), size=(df, C))]
    Ws = [w.astype(np.float32) for w in Ws]
    p = r.normal(size=(nh, d)).astype(np.float32)
    U = r.normal(size=(nh, S, d)).astype(np.float32)
    mask = (r.random((nh, S)) < 0.8).astype(np.uint8)
    mask[7] = 0
    dF = r.normal(size=(nh, df)).astype(np.float32)
    say("case: fusion forward / backward")
    fu = ann.Fusion(*Ws, heads=heads)
    F = fu.forward(_dev(p), _dev(U), _dev(mask))
    fu.backward(_dev(p), _dev(U), _dev(mask), _dev(dF))
    torch.cuda.synchronize()
    ref, cache = T.fusion_forward([w.astype(np.float64) for w in Ws], p, U, mask, heads)
    assert _rel(F.cpu().numpy(), ref) <= 1e-5
    assert (F.cpu().numpy()[7] == 0).all()
    grads = T.fusion_backward(cache, dF.astype(np.float64))
    for got, want in zip(fu.g, grads):
        assert _rel(got.cpu().numpy(), want) <= 1e-4


def test_train_step_hub_input_gradient_matches_oracle():
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    tq = synth.train_queries(ix["w"], 512)
    r = np.random.default_rng(2)
    labels = r.integers(0, hub_in.shape[0], size=tq.shape[0]).astype(np.int32)
    idx = r.permutation(tq.shape[0])[:256].astype(np.int32)
    say("case: train step with the hub input gradient")
    qt, ht = ann.Tower(*qp, in_scale=0.0625), ann.Tower(*hp)
    dx = torch.empty(hub_in.shape, dtype=torch.float32, device="cuda")
    ann.ann_train_step(qt, ht, _dev(tq), _dev(idx), _dev(labels), _dev(hub_in), 0.07, 1e-3, 0,
                       hub_in_grad=dx)
    torch.cuda.synchronize()
    eq, cq = T.tower_forward(qp, tq[idx].astype(np.float64), True, 0.0625)
    eh, ch = T.tower_forward(hp, hub_in.astype(np.float64), True)
    _, _, deh, _ = T.infonce(eq, eh, labels[idx], 0.07)
    ref = T.tower_backward_input(ch, deh, bf16=True)
    assert _rel(dx.cpu().numpy(), ref) <= 1e-3


@pytest.mark.parametrize("nh,e,s,Ls", [(96, 64, 16, (1, 4, 16, 48, 64)),
                                        (4096, 64, 8, (8, 32, 64)),
                                        (300, 128, 12, (5, 40)),
                                        (50, 16, 4, (2, 64))])
def test_hub_search_bit_exact_on_exact_embeddings(nh, e, s, Ls):
    # entries +-1/8: every embedding has norm 1 and every squared distance is
    # a multiple of 1/16, exact in FP32 in any summation order, so the
    # register-pool search must equal the oracle's search step for step
    ann = _ann()
    r = np.random.default_rng(nh + e)
    scale = 1.0 / np.sqrt(e) if e in (16, 64) else 1.0 / 8       # powers of two
    he = (r.choice([-1.0, 1.0], size=(nh, e)) * scale).astype(np.float32)
    qe = (r.choice([-1.0, 1.0], size=(200, e)) * scale).astype(np.float32)
    hg = oracle.hub_graph(he, s)
    start = oracle.hub_medoid(he)
    for L in Ls:
        say("case: hub search nh=%d e=%d s=%d L=%d" % (nh, e, s, L))
        b, d2, st, tr = ann.ann_hub_search(_dev(he), _dev(hg), _dev(qe), start, L, want_stats=True,
                                           trace_cap=512)
        torch.cuda.synchronize()
        ref = oracle.search(he, hg, qe, start, 1, L, trace_cap=512)
        assert (b.cpu().numpy() == ref["ids"][:, 0]).all(), L
        assert (d2.cpu().numpy().astype(np.float64) == ref["d2"][:, 0]).all(), L
        assert (st.cpu().numpy()[:, 0] == ref["ndc"]).all(), L
        assert (st.cpu().numpy()[:, 1] == ref["hops"]).all(), L
        assert (tr.cpu().numpy() == ref["trace"]).all(), L


def test_hub_search_on_trained_shapes_against_oracle_and_entry_select():
    # generic FP32 unit rows (tower outputs): equal to the oracle except at
    # certified near ties; ann_entry_select (which picks this search for
    # L_h <= 64) returns the same best hubs; above 64 it takes the base
    # search kernel, also checked against the oracle
    from tests.common import near_tie_certificate
    ix, km, hub_in, qp, hp = _setup()
    ann = _ann()
    qt, ht = ann.Tower(*qp), ann.Tower(*hp)
    hemb = ht.forward(_dev(hub_in))
    hg, hub_entry = ann.ann_navgraph_build(hemb, 8)
    qe_d = qt.forward(_dev(ix["q"]))
    torch.cuda.synchronize()
    he, qe, hgh = hemb.cpu().numpy(), qe_d.cpu().numpy(), hg.cpu().numpy()
    for L in (6, 24, 64):
        say("case: hub search on tower embeddings, L=%d" % L)
        b, _, _, tr = ann.ann_hub_search(hemb, hg, qe_d, hub_entry, L, trace_cap=512)
        b, tr = b.cpu().numpy(), tr.cpu().numpy()
        ref = oracle.search(he, hgh, qe, hub_entry, 1, L, trace_cap=512)
        for i in range(qe.shape[0]):
            if not (tr[i] == ref["trace"][i]).all():
                assert near_tie_certificate(he, hgh, qe[i], hub_entry, L, tr[i], ref["trace"][i]), i
            elif b[i] != ref["ids"][i, 0]:
                assert False, i
        model = ann.EntryModel(qt, hemb, hg, _dev(km["hub_ids"]), hub_entry, ix["medoid"], L_h=L)
        _, _, bh = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True)
        assert (bh.cpu().numpy() == b).all()
    say("case: entry select above the register pool (L_h = 96, base search kernel)")
    model = ann.EntryModel(qt, hemb, hg, _dev(km["hub_ids"]), hub_entry, ix["medoid"], L_h=96)
    _, _, bh = ann.ann_entry_select(model, _dev(ix["q"]), want_score=True)
    ref = oracle.search(he, hgh, qe, hub_entry, 1, 96)
    cos = qe.astype(np.float64) @ he.astype(np.float64).T
    bh = bh.cpu().numpy()
    for i in np.flatnonzero(bh != ref["ids"][:, 0]):
        assert abs(cos[i, bh[i]] - cos[i, ref["ids"][i, 0]]) <= 1e-5, i


def test_labels_dead_end_graph_by_hand():
    # the hand-traced graph of the oracle's pins: from E the widths 1 and 2
    # stall at a dead end, width 4 reaches the true neighbour with 7 distance
    # computations (width 8 would cost 8); from F width 1 reaches it with 4
    from tests.test_oracle_search import _dead_end_graph
    base, g, q = _dead_end_graph()
    say("case: labels on the hand-traced dead-end graph")
    lab, tab, flags = _ann().ann_make_labels(_dev(base), _dev(g), _dev(q), _dev(np.array([[0]], np.int32)),
                                             1, _dev(np.array([[0, 1]], np.int32)),
                                             _dev(np.array([1, 5, 4], np.int32)), [1, 2, 4, 8])
    torch.cuda.synchronize()
    assert tab.cpu().numpy().tolist() == [[7, 4]]
    assert lab.cpu().numpy().tolist() == [1] and flags.cpu().numpy().tolist() == [0]
    lab, tab, _ = _ann().ann_make_labels(_dev(base), _dev(g), _dev(q), _dev(np.array([[0]], np.int32)),
                                         1, _dev(np.array([[2, 0]], np.int32)),
                                         _dev(np.array([1, 5, 4], np.int32)), [1, 2])
    torch.cuda.synchronize()
    assert tab.cpu().numpy().tolist() == [[-1, -1]] and lab.cpu().numpy().tolist() == [2]


def test_labels_overflowing_the_visited_table_are_searched_again():
    # a random 64-regular graph on 9,000 integer points: at width 512 a
    # search visits almost every node, more ids than the first pass's table
    # (2^13 slots) holds, so the costs of those searches could count a node
    # twice; the library searches such queries again with 2^14 slots, and the
    # costs must then equal the oracle's exact distance counts
    ann = _ann()
    r = np.random.default_rng(33)
    n, d, R, nq = 9000, 32, 64, 20
    base = r.integers(0, 256, size=(n, d)).astype(np.float32)
    g = np.empty((n, R), np.int32)
    for v in range(n):
        nb = r.choice(n - 1, R, replace=False)
        g[v] = np.where(nb >= v, nb + 1, nb)
    q = r.integers(0, 256, size=(nq, d)).astype(np.float32)
    truth, _ = oracle.knn(base, q, 10)
    hubs = np.array([11, 222, 3333, 4444], np.int32)
    cand = np.tile(np.arange(4, dtype=np.int32), (nq, 1))
    ladder = [10, 512]
    say("case: labels with visited-table overflow (oracle)")
    ref_lab, ref_tab = oracle.make_labels(base, g, q, truth, cand, hubs, ladder, 10)
    say("case: labels with visited-table overflow (gpu)")
    lab, tab, flags = ann.ann_make_labels(_dev(base), _dev(g), _dev(q), _dev(truth), 10, _dev(cand),
                                          _dev(hubs), ladder)
    torch.cuda.synchronize()
    lab, tab, flags = lab.cpu().numpy(), tab.cpu().numpy(), flags.cpu().numpy()
    # the first pass's table does overflow here
    plan = ann.make_plan(**dict(ann.default_plan(n, d, R, 512).as_dict(), filter=ann.ANN_FILTER_ID32,
                                visited_log2=13))
    st = ann.ann_search(_dev(base), _dev(g), _dev(q), _dev(np.full(nq, hubs[0], np.int32)), 0, 10,
                        512, plan=plan)[2].cpu().numpy()
    say("first-pass overflows at width 512: %d of %d; final flags %d" %
        (int((st[:, 3] & 1).sum()), nq, int((flags & 1).sum())))
    assert (st[:, 3] & 1).sum() > 0
    assert (flags == 0).all()
    assert (tab == ref_tab).all()
    assert (lab == ref_lab).all()


def test_trained_entry_beats_untrained_towers_and_medoid():
    # What the trained network gains over the method without it (the paper's
    # ablation without the learned part): the same index, hubs, features and
    # labels, one entry model trained and one left at its initial weights,
    # and the plain method's medoid entry, compared on held-out test queries
    # at fixed beam widths.  200,000 points of the 1M x 128 recipe (256
    # components), 256 hubs, 30,000 training queries, 2,000 test queries.
    ann = _ann()
    from paper_2506_15986_amd import gate
    w = synth.scaled(synth.WORKLOADS["sift1m"], n=200_000, n_queries=2_000, n_train=30_000)
    dev = torch.device("cuda:0")
    say("case: gain test: data, graph, hubs, labels (200k x 128)")
    bd = torch.from_numpy(synth.base(w)).to(dev)
    qd = torch.from_numpy(synth.queries(w)).to(dev)
    tq = torch.from_numpy(synth.train_queries(w)).to(dev)
    index = gate.build_index(bd, 128, 32, 1.2)
    data = gate.prepare_gate(index, tq, w, n_hubs=256, log=say)
    say("case: gain test: trained and untrained towers")
    trained = gate.train_gate(index, data, tq, w, epochs=20, log=say)
    untrained = gate.train_gate(index, data, tq, w, train=False, log=say)
    gt = ann.ann_gt_knn(bd, qd, 10)[0].cpu().numpy()
    rows = {}
    for name, ent in (("trained", trained.select(qd)[0]), ("untrained", untrained.select(qd)[0]),
                      ("medoid", None)):
        for L in (32, 64, 128):
            ids, _, st, _ = index.search(qd, L, 10, ent)
            rec = float((ids.cpu().numpy()[:, :, None] == gt[:, None, :]).any(-1).mean())
            rows[name, L] = (rec, float(st[:, 0].float().mean().item()))
    say("gain test (recall@10, mean ndc): %s" % rows)
    say("held-out label agreement: trained %.3f, untrained %.3f" %
        (trained.info["val_top1"], untrained.info["val_top1"]))
    assert trained.info["val_top1"] >= untrained.info["val_top1"] + 0.2
    for L in (32, 64, 128):
        rt = rows["trained", L][0]
        assert rt >= rows["untrained", L][0] + 0.2, L
        assert rt >= rows["medoid", L][0] + 0.2, L
    # the trained entry reaches at L = 64 at least the recall that the other
    # two do not reach at twice that width
    assert rows["trained", 64][0] > max(rows["untrained", 128][0], rows["medoid", 128][0])
