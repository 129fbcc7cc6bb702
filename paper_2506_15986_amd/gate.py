"""Index and entry-model construction for the GATE query path, composed from
the libann entry points (every step runs in the library's kernels; this
module only sequences the calls and holds the device tensors).

    index = build_index(base, knn_k=128, R=32, alpha=1.2)
    gate = build_gate(index, train_queries, workload)
    entries = gate.select(queries)            # query tower + hub-graph search
    ids, dist, stats, _ = index.search(queries, L, k, entries)
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import ann, synth


@dataclasses.dataclass
class Index:
    base: torch.Tensor
    graph: torch.Tensor
    medoid: int
    bridges: tuple
    R: int
    build_s: float

    @property
    def n(self):
        return self.base.shape[0]

    @property
    def dim(self):
        return self.base.shape[1]

    def search(self, queries, L, k, entry_ids=None, plan=None, out=None, ws=None):
        nq = queries.shape[0]
        dev = queries.device
        kk = k if torch.is_tensor(k) else torch.full((nq,), int(k), dtype=torch.int32, device=dev)
        LL = L if torch.is_tensor(L) else torch.full((nq,), int(L), dtype=torch.int32, device=dev)
        if plan is None:
            Lmax = int(L) if not torch.is_tensor(L) else int(LL.max().item())
            plan = ann.default_plan(self.n, self.dim, self.R, Lmax)
        return ann.ann_search(self.base, self.graph, queries, entry_ids, self.medoid, kk, LL,
                              k_max=int(k) if not torch.is_tensor(k) else None, plan=plan,
                              out=out, ws=ws)


def build_index(base: torch.Tensor, knn_k: int = 128, R: int = 32, alpha: float = 1.2,
                partitions: int = 0, overlap: int = 2, w: synth.Workload | None = None,
                log=None) -> Index:
    """The proximity graph: all-pairs exact kNN candidates, or with
    partitions > 0 candidates from overlapping groups: Lloyd k-means
    (`partitions` clusters, 10 steps, seeded from the workload) gives the
    hubs; each point lists its `overlap` nearest hubs, the first being its
    home group, and its candidates are the exact knn_k nearest among the
    points that list its home group (computed a few groups per call, with a
    `log` line after each).  Then alpha pruning, medoid, repair."""
    t = time.time()
    if partitions > 0:
        n = base.shape[0]
        init = torch.from_numpy(synth.kmeans_init(w, n, partitions)).to(base.device)
        hub_ids, _, _, _ = ann.ann_select_hubs(base, partitions, 10, init)
        hubs = base[hub_ids.long()].contiguous()
        groups = torch.empty((n, overlap), dtype=torch.int32, device=base.device)
        step = 1 << 20
        for s in range(0, n, step):
            ids, _ = ann.ann_gt_knn(hubs, base[s:s + step], overlap)
            groups[s:s + step] = ids
        sizes = ann.group_sizes(groups.cpu().numpy(), partitions)
        cand = torch.empty((n, knn_k), dtype=torch.int32, device=base.device)
        cd2 = torch.empty((n, knn_k), dtype=torch.float64, device=base.device)
        step = 4
        for g0 in range(0, partitions, step):
            ann.ann_group_candidates(base, knn_k, groups, partitions, g0,
                                     min(partitions, g0 + step), cand, cd2, sizes=sizes)
            if log:
                log("  candidate lists: groups %d..%d of %d done (%.1fs)" %
                    (g0, min(partitions, g0 + step) - 1, partitions, time.time() - t))
        graph, med, bridges = ann.ann_graph_from_candidates(base, cand, cd2, R, alpha)
        del cand, cd2
    else:
        graph, med, bridges = ann.ann_build_graph(base, knn_k, R, alpha)
    torch.cuda.synchronize()
    return Index(base, graph, med, bridges, R, time.time() - t)


def build_index_nsg(base: torch.Tensor, knn_k: int = 128, R: int = 32, L_build: int = 128,
                    path: int = 0, chunk: int = 1 << 18, log=None) -> Index:
    """NSG-style proximity graph (the base index the paper assumes): exact
    kNN lists (knn_k, self excluded); every base point searched for from the
    medoid over the kNN graph's first min(knn_k, 64) columns with beam width
    L_build (the whole pool kept, and with path > 0 also the first `path`
    nodes the search expanded); these and the kNN list merged per point
    (ann_merge_candidates); MRNG pruning (alpha = 1) to R - 2, medoid and
    repair (ann_graph_from_candidates)."""
    t = time.time()
    n, dim = base.shape
    if L_build + path + knn_k > 1024:
        raise ValueError("L_build + path + knn_k must be <= 1024")
    knn_ids, _ = ann.ann_gt_knn(base, base, knn_k, exclude_self=True)
    if log:
        log("  nsg: kNN %d lists (%.1fs)" % (knn_k, time.time() - t))
    g0 = knn_ids[:, :min(knn_k, 64)].contiguous()
    med = ann.ann_medoid(base)
    plan = ann.default_plan(n, dim, g0.shape[1], L_build)
    pool = torch.empty((n, L_build + path), dtype=torch.int32, device=base.device)
    ws = ann.workspace("search", n, dim, min(chunk, n), device=base.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        ids, _, _, tr = ann.ann_search(base, g0, base[s:e], None, med, L_build, L_build,
                                       plan=plan, want_stats=False, trace_cap=path, ws=ws)
        pool[s:e, :L_build] = ids
        if path:
            pool[s:e, L_build:] = tr
        del ids, tr
    torch.cuda.synchronize()
    del ws, g0
    if log:
        log("  nsg: %d search pools of width %d (%.1fs)" % (n, L_build, time.time() - t))
    cand, cd2 = ann.ann_merge_candidates(base, pool, knn_ids)
    del pool
    graph, med2, bridges = ann.ann_graph_from_candidates(base, cand, cd2, R, 1.0)
    del cand, cd2
    torch.cuda.synchronize()
    ix = Index(base, graph, med2, bridges, R, time.time() - t)
    # how many pruned-graph edges (slots before the two repair slots) came
    # from the search pools alone, not from the kNN lists
    edges = from_pool = 0
    for s in range(0, n, 1 << 16):
        g = graph[s:s + (1 << 16), :R - 2]
        inl = (g[:, :, None] == knn_ids[s:s + (1 << 16), None, :]).any(-1)
        edges += int((g >= 0).sum().item())
        from_pool += int(((g >= 0) & ~inl).sum().item())
    ix.edge_stats = dict(edges=edges, from_pool_only=from_pool)
    del knn_ids
    return ix


@dataclasses.dataclass
class Gate:
    qtower: ann.Tower
    htower: ann.Tower
    hub_ids: torch.Tensor
    hub_in: torch.Tensor
    hub_emb: torch.Tensor
    hub_graph: torch.Tensor
    hub_entry: int
    model: ann.EntryModel
    info: dict

    def select(self, queries, out=None, want_score=False):
        return ann.ann_entry_select(self.model, queries, want_score=want_score, out=out)


def nearest_hub_entries(index: Index, hub_ids: torch.Tensor, queries: torch.Tensor):
    """Ablation without learning: entry = the hub nearest the query by L2."""
    hv = ann.ann_hub_input(index.base, hub_ids)
    ids, _ = ann.ann_gt_knn(hv, queries, 1)
    return hub_ids[ids[:, 0].long()].contiguous()


@dataclasses.dataclass
class GateData:
    """Everything the entry model is trained from: hubs, hub-tower inputs and
    the per-query labels (with the nearest-hub candidates they were chosen
    among)."""
    hub_ids: torch.Tensor
    hub_in: torch.Tensor
    labels: torch.Tensor
    cand: torch.Tensor
    scale: float
    info: dict
    nn: torch.Tensor | None = None     # each training query's nearest base point


def prepare_gate(index: Index, train_q: torch.Tensor, w: synth.Workload, n_hubs: int = 1024,
                 kmeans_iters: int = 20, M: int = 8,
                 ladder=(10, 16, 24, 32, 48, 64, 96, 128, 192, 256), hubs: str = "lloyd",
                 hbkm_lambda: float = 0.0, hbkm_iters: int = 10, log=print) -> GateData:
    """Hubs (Definition 3 on Lloyd k-means, or with hubs="hbkm" on the
    hierarchical balanced k-means of Algorithm 2 with k = n_hubs^(1/2), two
    levels), hub topology features, hub-tower inputs and the training
    labels."""
    base, dev = index.base, index.base.device
    n, d = base.shape
    info = {}
    t = time.time()
    if hubs == "hbkm":
        k = int(round(math.sqrt(n_hubs)))
        if k * k != n_hubs:
            raise ValueError("HBKM hubs need n_hubs = k^2 (got %d)" % n_hubs)
        hub_ids, cen, assign = ann.ann_select_hubs_hbkm(base, k, 2, hbkm_lambda, hbkm_iters)
        steps = 2 * hbkm_iters
        sizes = torch.bincount(assign.long(), minlength=n_hubs).double()
        info["hbkm"] = dict(k=k, levels=2, lam=hbkm_lambda, iters=hbkm_iters,
                            size_objective=float(((sizes - n / n_hubs) ** 2).sum().item()),
                            size_min=int(sizes.min().item()), size_max=int(sizes.max().item()))
    else:
        init = torch.from_numpy(synth.kmeans_init(w, n, n_hubs)).to(dev)
        hub_ids, cen, assign, steps = ann.ann_select_hubs(base, n_hubs, kmeans_iters, init)
        sizes = torch.bincount(assign.long(), minlength=n_hubs).double()
        info["size_objective"] = float(((sizes - n / n_hubs) ** 2).sum().item())
    torch.cuda.synchronize()
    info["kmeans_steps"] = steps
    info["hubs_s"] = time.time() - t
    log("hubs (%s): %d steps, %.1fs" % (hubs, steps, info["hubs_s"]))

    t = time.time()
    # inputs scaled by a power of two into [-1, 1] (exact in BF16)
    scale = ann.input_scale(ann.ann_max_abs(base))
    info["input_scale"] = scale
    feat, _ = ann.ann_hub_features(base, index.graph, index.medoid, hub_ids, assign, cen)
    hub_in = ann.ann_hub_input(base, hub_ids, feat, vec_scale=scale)
    hub_vec = ann.ann_hub_input(base, hub_ids)
    torch.cuda.synchronize()
    info["features_s"] = time.time() - t

    t = time.time()
    truth, _ = ann.ann_gt_knn(base, train_q, 10)
    cand, _ = ann.ann_gt_knn(hub_vec, train_q, M)
    labels, table, flags = ann.ann_make_labels(base, index.graph, train_q, truth, 10, cand, hub_ids,
                                               list(ladder))
    torch.cuda.synchronize()
    info["labels_s"] = time.time() - t
    tab = table.cpu().numpy()
    info["labels_reached"] = float((tab >= 0).any(axis=1).mean())
    info["label_is_nearest_hub"] = float((labels.cpu().numpy() == cand[:, 0].cpu().numpy()).mean())
    info["label_flags"] = int((flags.cpu().numpy() != 0).sum())
    log("labels: %.1fs, reached %.3f, nearest-hub agreement %.3f" %
        (info["labels_s"], info["labels_reached"], info["label_is_nearest_hub"]))
    return GateData(hub_ids, hub_in, labels, cand, scale, info, nn=truth[:, 0].contiguous())


def train_gate(index: Index, data: GateData, train_q: torch.Tensor, w: synth.Workload,
               hidden: int = 128, dout: int = 64, epochs: int = 20, batch: int = 1024,
               lr: float = 1e-3, tau: float = 0.07, s: int = 16, L_h: int = 32,
               theta: float = -math.inf, train: bool = True, holdout: float = 0.1,
               init: str = "random", tune_L_h: bool = True, objective: str = "labels",
               t_pos: int = 3, t_neg: int = 15, queue_hubs: int = 64, queue_P: int = 16,
               queue_N: int = 48, select_best: bool = False, val_every: int = 1,
               fusion: bool = False, fusion_heads: int = 4,
               fusion_dk: int = 16, fusion_df: int = 64, log=print) -> Gate:
    """Trains the towers on the first (1 - holdout) of the training queries
    (contrastive loss, Adam), embeds the hubs, builds the navigation graph and
    reports top-1 label agreement on the trained and the held-out queries.
    With select_best (labels objective), the entry model's held-out label
    agreement is measured every val_every epochs and the towers of the best
    epoch are kept: `epochs` is then a budget, not a fixed count.

    objective "labels": each query against all hubs with its label hub as the
    positive.  "queues": Definition 4 queues (hop counts from every hub to
    each query's nearest neighbour; positives within t_pos hops of the hub's
    closest query, negatives t_neg or more hops beyond it) and Eq. 4 read
    hub-anchored, queue_hubs hubs per step with queue_P positives and
    queue_N negatives each; as many steps per epoch as fill the training
    queries once (queue_hubs * (queue_P + queue_N) query rows per step).

    fusion: the hub tower reads [hub vector | F | features] with F the Eq. 3
    fusion embedding of the hub vector over its topology tokens (the relative
    positions x_w - x_hub of its graph neighbours, scaled like the vectors;
    empty slots masked), trained with the towers through the hub tower's input
    gradient (labels objective)."""
    dev = index.base.device
    d = index.dim
    n_hubs = data.hub_ids.shape[0]
    info = dict(data.info)
    hub_in, labels = data.hub_in, data.labels
    fu = None
    if fusion:
        p_vec, U, tok_mask = ann.ann_fusion_tokens(index.base, index.graph, data.hub_ids,
                                                   data.scale)
        C = fusion_heads * fusion_dk
        fw = synth.tower_init(w, [(C, d), (C, d), (C, d), (fusion_df, C)], salt=3)
        fu = ann.Fusion(fw[0], fw[2], fw[4], fw[6], heads=fusion_heads, device=dev)
        feat = hub_in[:, d:]
        hub_in = torch.cat([hub_in[:, :d], fu.forward(p_vec, U, tok_mask), feat], dim=1).contiguous()
    qp = synth.tower_init(w, [(hidden, d), (dout, hidden)])
    hp = synth.tower_init(w, [(hidden, hub_in.shape[1]), (dout, hidden)])
    if init == "tied":
        qp, hp = tied_init(qp, hub_in.cpu().numpy(), d)
    qt = ann.Tower(*qp, device=dev, in_scale=data.scale)
    ht = ann.Tower(*hp, device=dev)
    t = time.time()
    nt_all = train_q.shape[0]
    n_hold = int(round(holdout * nt_all))
    nt = nt_all - n_hold
    step = 0
    losses = []
    nb = ann.ann_train_workspace_size(batch, n_hubs, d, hub_in.shape[1], hidden, dout)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    if train and objective == "queues":
        H = ann.ann_hop_table(index.graph, data.hub_ids, data.nn[:nt].contiguous())
        # Definition 4 queues (hub-major lists with offsets), built in the library
        pos_off_d, pos_q, neg_off_d, neg_q = ann.ann_make_queues(H, t_pos, t_neg)
        pos_off, neg_off = pos_off_d.cpu().numpy(), neg_off_d.cpu().numpy()
        eligible = np.flatnonzero((np.diff(pos_off) > 0) & (np.diff(neg_off) > 0))
        info.update(queue_hubs_eligible=int(eligible.size),
                    queue_pos_mean=float(np.diff(pos_off)[eligible].mean()) if eligible.size else 0.0,
                    queue_neg_mean=float(np.diff(neg_off)[eligible].mean()) if eligible.size else 0.0,
                    t_pos=t_pos, t_neg=t_neg)
        del H
        rows = queue_hubs * (queue_P + queue_N)
        spe = max(1, -(-nt // rows))
        nb = ann.ann_train_hub_workspace_size(queue_hubs, queue_P, queue_N, d, hub_in.shape[1], hidden,
                                              dout)
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
        for ep in range(epochs):
            for _ in range(spe):
                step += 1
                hb, pp, nn = synth.queue_batch(w, step, eligible, pos_off, neg_off, queue_hubs,
                                               queue_P, queue_N)
                qi = torch.cat([pos_q[torch.from_numpy(pp).to(dev)],
                                neg_q[torch.from_numpy(nn).to(dev)]], dim=1)
                loss, _, _ = ann.ann_train_step_hub(qt, ht, train_q, qi.reshape(-1).to(torch.int32),
                                                    torch.from_numpy(hb.astype(np.int32)).to(dev),
                                                    queue_P, queue_N, hub_in, tau, lr, step, ws=ws)
            losses.append(loss.item())
        log("queues: %d of %d hubs with both queues, %.0f positives / %.0f negatives per hub" %
            (eligible.size, n_hubs, info["queue_pos_mean"], info["queue_neg_mean"]))
    elif train and fu is not None:
        dx = torch.empty_like(hub_in)
        fd = fu.df
        for ep in range(epochs):
            order = torch.from_numpy(synth.batch_order(w, nt, ep).astype(np.int32)).to(dev)
            for b0 in range(0, nt - batch + 1, batch):
                step += 1
                hub_in[:, d:d + fd] = fu.forward(p_vec, U, tok_mask)
                loss, _, _ = ann.ann_train_step(qt, ht, train_q, order[b0:b0 + batch], labels, hub_in,
                                                tau, lr, step, ws=ws, hub_in_grad=dx)
                fu.backward(p_vec, U, tok_mask, dx[:, d:d + fd].contiguous())
                fu.adam(lr, step)
            losses.append(loss.item())
        hub_in[:, d:d + fd] = fu.forward(p_vec, U, tok_mask)
    elif train:
        best = (-1.0, -1, None)
        val_curve = []
        for ep in range(epochs):
            order = torch.from_numpy(synth.batch_order(w, nt, ep).astype(np.int32)).to(dev)
            for b0 in range(0, nt - batch + 1, batch):
                step += 1
                loss, _, _ = ann.ann_train_step(qt, ht, train_q, order[b0:b0 + batch], labels, hub_in,
                                                tau, lr, step, ws=ws)
            losses.append(loss.item())
            if select_best and n_hold and (ep % val_every == val_every - 1 or ep == epochs - 1):
                # held-out label agreement of the entry model as it stands
                hemb = ht.forward(hub_in)
                hg, he = ann.ann_navgraph_build(hemb, s)
                mdl = ann.EntryModel(qt, hemb, hg, data.hub_ids, he, index.medoid, L_h=L_h,
                                     theta=theta)
                _, _, bh = ann.ann_entry_select(mdl, train_q[nt:], want_score=True)
                acc = float((bh == labels[nt:]).float().mean().item())
                val_curve.append((ep + 1, round(acc, 4)))
                if acc > best[0]:
                    best = (acc, ep + 1, [t.clone() for t in qt.params() + ht.params()])
                del mdl, hemb, hg
        if best[2] is not None:
            for dst, src in zip(qt.params() + ht.params(), best[2]):
                dst.copy_(src)
            qt.sync()
            ht.sync()
            info.update(selected_epoch=best[1], val_curve=val_curve)
            log("training: held-out agreement best after epoch %d of %d (%.3f)" %
                (best[1], epochs, best[0]))
    torch.cuda.synchronize()
    info.update(train_s=time.time() - t, train_steps=step, hidden=hidden, dout=dout, objective=objective,
                fusion=dict(heads=fusion_heads, dk=fusion_dk, df=fusion_df) if fusion else None,
                epochs=epochs, lr=lr, tau=tau, holdout=n_hold,
                loss_per_epoch=[round(x, 4) for x in losses])
    if losses:
        log("training: %d steps, %.1fs, loss %.3f -> %.3f" % (step, info["train_s"], losses[0],
                                                              losses[-1]))
    hemb = ht.forward(hub_in)
    hg, hub_entry = ann.ann_navgraph_build(hemb, s)
    model = ann.EntryModel(qt, hemb, hg, data.hub_ids, hub_entry, index.medoid, L_h=L_h,
                           theta=theta)
    if tune_L_h:
        info["L_h"] = model.tune_L_h(train_q[:min(nt, 10000)])
        info["L_h_agreement"] = model.L_h_rates
    info["hub_plan"] = model.tune_hub_plan(train_q[:min(nt, 10000)]).as_dict()
    # label agreement: does the query tower pick the label hub?
    m = min(nt, 10000)
    _, _, bh = ann.ann_entry_select(model, train_q[:m], want_score=True)
    info["train_top1"] = float((bh == labels[:m]).float().mean().item())
    if n_hold:
        _, _, bh = ann.ann_entry_select(model, train_q[nt:], want_score=True)
        info["val_top1"] = float((bh == labels[nt:]).float().mean().item())
        info["val_nearest_hub_top1"] = float((data.cand[nt:, 0] == labels[nt:]).float().mean().item())
    log("entry model: top-1 agreement with labels: train %.3f, held-out %s" %
        (info["train_top1"], "%.3f" % info["val_top1"] if n_hold else "-"))
    return Gate(qt, ht, data.hub_ids, hub_in, hemb, hg, hub_entry, model, info)


def tune_theta(index: Index, g: Gate, queries: torch.Tensor, truth: torch.Tensor, L: int,
               k: int = 10, quantiles=(0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.3, 0.5)):
    """The medoid fallback's threshold theta (entries whose best hub has a
    cosine below theta start at the medoid): tried at -inf and at quantiles
    of the queries' best-hub cosines, each judged by recall@k at beam width L
    against `truth` (the queries' exact top-k); the best recall wins, ties to
    the smaller theta (fewer fallbacks).  Sets g.model's theta and returns
    (theta, [(theta, recall, fallbacks), ...])."""
    m = g.model
    old = float(m.c.theta)
    m.c.theta = -math.inf
    _, sc, _ = ann.ann_entry_select(m, queries, want_score=True)
    cands = [-math.inf] + sorted(set(float(x) for x in
                                     torch.quantile(sc.double(), torch.tensor(
                                         list(quantiles), dtype=torch.float64,
                                         device=sc.device)).tolist()))
    tr = truth[:, :k].cpu().numpy()
    rows, best = [], None
    for th in cands:
        m.c.theta = th
        ent = ann.ann_entry_select(m, queries)[0]
        ids = index.search(queries, L, k, ent)[0].cpu().numpy()
        rec = float((ids[:, :k, None] == tr[:, None, :]).any(-1).mean())
        fb = int((ent == index.medoid).sum().item())
        rows.append((th, round(rec, 5), fb))
        if best is None or rec > best[1]:
            best = (th, rec)
    m.c.theta = best[0] if best is not None else old
    return float(m.c.theta), rows


def tied_init(qp, hub_in: np.ndarray, d: int):
    """Siamese start for the two towers: the hub tower's weights on the hub
    vector equal the query tower's, its weights on the topology features start
    at zero, and the first-layer bias centres the (scaled) inputs on the mean
    hub vector.  A query and a hub vector then get the same embedding, so
    cosine order starts from the geometry of the data and training adjusts
    it.  qp: the query tower's (W1, b1, W2, b2) as drawn."""
    W1, b1, W2, b2 = [np.asarray(a, np.float32) for a in qp]
    centre = hub_in[:, :d].astype(np.float64).mean(0)
    b1c = (b1.astype(np.float64) - W1.astype(np.float64) @ centre).astype(np.float32)
    W1h = np.concatenate([W1, np.zeros((W1.shape[0], hub_in.shape[1] - d), np.float32)], 1)
    return (W1, b1c, W2, b2), (W1h, b1c.copy(), W2.copy(), b2.copy())


def build_gate(index: Index, train_q: torch.Tensor, w: synth.Workload, n_hubs: int = 1024,
               kmeans_iters: int = 20, M: int = 8,
               ladder=(10, 16, 24, 32, 48, 64, 96, 128, 192, 256), data: GateData | None = None,
               log=print, **train_kw) -> Gate:
    if data is None:
        data = prepare_gate(index, train_q, w, n_hubs, kmeans_iters, M, ladder, log=log)
    return train_gate(index, data, train_q, w, log=log, **train_kw)


def save_state(path: str, index: Index, gate: Gate | None, extra: dict) -> None:
    """Writes the built index and entry model (arrays as .npy, scalars as
    JSON) so that a later process can serve without rebuilding."""
    import json
    import os
    os.makedirs(path, exist_ok=True)
    np.save(os.path.join(path, "graph.npy"), index.graph.cpu().numpy())
    meta = dict(extra, medoid=int(index.medoid), bridges=list(index.bridges), R=int(index.R),
                build_s=float(index.build_s), gate=gate is not None)
    if gate is not None:
        qt = gate.qtower
        for name, t in (("qW1", qt.W1), ("qb1", qt.b1), ("qW2", qt.W2), ("qb2", qt.b2),
                        ("hub_ids", gate.hub_ids), ("hub_emb", gate.hub_emb),
                        ("hub_graph", gate.hub_graph)):
            np.save(os.path.join(path, name + ".npy"), t.cpu().numpy())
        meta.update(in_scale=qt.in_scale, hub_entry=int(gate.hub_entry),
                    L_h=int(gate.model.c.L_h), theta=float(gate.model.c.theta), info=gate.info,
                    hub_plan=gate.model.c.hub_plan.as_dict())
    with open(os.path.join(path, "meta.json"), "w") as f:
        json.dump(meta, f)


def load_state(path: str, base: torch.Tensor):
    """Inverse of save_state: returns (index, gate or None, meta)."""
    import json
    import os
    dev = base.device
    with open(os.path.join(path, "meta.json")) as f:
        meta = json.load(f)
    ld = lambda name: torch.from_numpy(np.load(os.path.join(path, name + ".npy"))).to(dev)
    index = Index(base, ld("graph").contiguous(), int(meta["medoid"]), tuple(meta["bridges"]),
                  int(meta["R"]), float(meta["build_s"]))
    gate = None
    if meta["gate"]:
        qt = ann.Tower(ld("qW1"), ld("qb1"), ld("qW2"), ld("qb2"), device=dev,
                       in_scale=float(meta["in_scale"]))
        hub_ids, hemb, hg = ld("hub_ids"), ld("hub_emb"), ld("hub_graph")
        model = ann.EntryModel(qt, hemb, hg, hub_ids, int(meta["hub_entry"]), index.medoid,
                               L_h=int(meta["L_h"]), theta=float(meta["theta"]),
                               hub_plan=ann.make_plan(**meta["hub_plan"]) if meta.get("hub_plan")
                               else None)
        gate = Gate(qt, None, hub_ids, None, hemb, hg, int(meta["hub_entry"]), model,
                    dict(meta.get("info", {})))
    return index, gate, meta
