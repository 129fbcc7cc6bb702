"""Pins for the oracle's best-first beam search (Algorithm 1 reading), its
label-search extension, and the hub-graph entry selection."""
import math

import numpy as np
import pytest

import oracle
from paper_2506_15986_amd import synth


def path_graph(n):
    """x_m = m on a line; node m links to m-1 then m+1 (slot order)."""
    base = np.zeros((n, 3), np.float32)
    base[:, 0] = np.arange(n)
    g = -np.ones((n, 2), np.int32)
    for m in range(n):
        s = 0
        if m > 0:
            g[m, s] = m - 1
            s += 1
        if m < n - 1:
            g[m, s] = m + 1
    return base, g


@pytest.mark.parametrize("i,j", [(5, 12), (12, 5), (3, 4), (20, 2)])
def test_path_graph_hops_and_ndc_closed_form(i, j):
    n = 30
    base, g = path_graph(n)
    r = oracle.search(base, g, base[j:j + 1], i, 1, 1)
    assert r["ids"][0, 0] == j
    assert r["hops"][0] == abs(i - j) + 1
    assert r["ndc"][0] == abs(i - j) + 3


@pytest.mark.parametrize("entry_rank_in", [True, False])
def test_complete_graph(entry_rank_in):
    n, d, k, L = 40, 4, 5, 8
    r = np.random.default_rng(3)
    base = r.normal(size=(n, d)).astype(np.float32)
    q = r.normal(size=(1, d)).astype(np.float32)
    g = np.array([[w for w in range(n) if w != v] for v in range(n)], np.int32)
    truth, _ = oracle.knn(base, q, n)
    entry = int(truth[0, 2]) if entry_rank_in else int(truth[0, -1])
    res = oracle.search(base, g, q, entry, k, L)
    assert res["ndc"][0] == n
    assert res["ids"][0].tolist() == truth[0, :k].tolist()
    assert res["hops"][0] == (L if entry_rank_in else L + 1)


def _tiny_graph(n=600):
    w = synth.scaled(synth.WORKLOADS["tiny"], n=n, n_queries=12)
    base = synth.base(w)
    q = synth.queries(w)
    g, med, *_ = oracle.build_graph(base, knn_k=64, R=16, alpha=1.2)
    return base, q, g, med


def test_beam_width_at_least_n_gives_exact_knn():
    base, q, g, med = _tiny_graph()
    n = base.shape[0]
    truth, td2 = oracle.knn(base, q, 10)
    r = oracle.search(base, g, q, med, 10, n)
    assert (r["ids"] == truth).all()
    assert (r["d2"] == td2).all()
    # the graph is strongly connected, so every node got visited
    assert (r["ndc"] == n).all()


def test_results_sorted_visited_closed_and_counts():
    base, q, g, med = _tiny_graph()
    n = base.shape[0]
    r = oracle.search(base, g, q, med, 10, 32, trace_cap=4096, want_visited=True)
    for i in range(q.shape[0]):
        ids, dd = r["ids"][i], r["d2"][i]
        keys = list(zip(dd.tolist(), ids.tolist()))
        assert keys == sorted(keys)
        vis = r["visited"][i].astype(bool)
        expanded = [p for p in r["trace"][i] if p >= 0]
        assert len(expanded) == r["hops"][i] and len(set(expanded)) == len(expanded)
        for p in expanded:
            nb = g[p][g[p] >= 0]
            assert vis[nb].all()                    # closed under expansion
        assert vis.sum() == r["ndc"][i] <= n
        assert r["hops"][i] <= r["ndc"][i]
        # every result is a visited node and its distance is the exact one
        for t in range(10):
            assert vis[ids[t]]
            assert dd[t] == oracle.sqdist(q[i], base[ids[t]])
        # the pool keeps the L best keys ever offered, so the result is the k
        # smallest keys of the visited set
        vk = sorted((oracle.sqdist(q[i], base[v]), int(v)) for v in np.where(vis)[0])
        assert [v for _, v in vk[:10]] == ids.tolist()


def test_per_query_k_and_L_padding():
    base, q, g, med = _tiny_graph()
    ks = np.array([1, 5, 10] * 4)[:q.shape[0]]
    Ls = np.array([10, 20, 40] * 4)[:q.shape[0]]
    r = oracle.search(base, g, q, med, ks, Ls, k_max=10)
    for i in range(q.shape[0]):
        assert (r["ids"][i, ks[i]:] == -1).all()
        assert np.isinf(r["d2"][i, ks[i]:]).all()
        one = oracle.search(base, g, q[i:i + 1], med, int(ks[i]), int(Ls[i]))
        assert (one["ids"][0] == r["ids"][i, :ks[i]]).all()


def test_labels_complete_graph_closed_form():
    # on the complete graph the first expansion evaluates every node, so every
    # (query, hub) costs exactly n at the first width and the label is the
    # smallest hub index among the candidates
    n, d = 40, 4
    r = np.random.default_rng(7)
    base = r.normal(size=(n, d)).astype(np.float32)
    q = r.normal(size=(5, d)).astype(np.float32)
    g = np.array([[w for w in range(n) if w != v] for v in range(n)], np.int32)
    truth, _ = oracle.knn(base, q, 10)
    hubs = np.array([30, 5, 17, 22], np.int32)
    cand = np.array([[2, 0, 3, 1]] * 5, np.int32)
    label, table = oracle.make_labels(base, g, q, truth, cand, hubs, [10, 20], 10)
    assert (table == n).all()
    assert (label == 0).all()


def test_labels_invariants_and_full_width():
    base, q, g, med = _tiny_graph()
    n = base.shape[0]
    truth, _ = oracle.knn(base, q, 10)
    hubs = np.array([0, 50, 100, 150, 200, 250, 300, 350], np.int32)
    cand = np.tile(np.arange(len(hubs), dtype=np.int32), (q.shape[0], 1))
    label, table = oracle.make_labels(base, g, q, truth, cand, hubs, [10, 32, n], 10)
    # a width >= n explores the strongly connected graph completely, so every
    # pair reaches the exact top-10; a cost can never be below the hit count
    assert (table >= 10).all() and (table <= n).all()
    for i in range(q.shape[0]):
        best = min((table[i, m], m) for m in range(len(hubs)))
        assert label[i] == best[1]


# ---------------------------------------------------------------- hub graph / entry
def _unit(r, n, e):
    x = r.normal(size=(n, e))
    return (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)


def test_hub_graph_is_top_cosine():
    # on unit vectors the squared-L2 order is the cosine order
    r = np.random.default_rng(4)
    emb = _unit(r, 64, 16)
    s = 6
    hg = oracle.hub_graph(emb, s)
    cos = emb.astype(np.float64) @ emb.astype(np.float64).T
    for i in range(64):
        row = hg[i].tolist()
        assert i not in row and len(set(row)) == s
        vals = [cos[i, j] for j in row]
        assert all(a >= b - 1e-12 for a, b in zip(vals, vals[1:]))
        others = [cos[i, j] for j in range(64) if j != i and j not in row]
        assert max(others) <= min(vals) + 1e-12


def test_entry_select_full_width_is_exact_argmax_and_theta_fallback():
    r = np.random.default_rng(5)
    nh, e = 48, 16
    hemb = _unit(r, nh, e)
    qemb = _unit(r, 30, e)
    hg = oracle.hub_graph(hemb, 6)
    hub_ids = np.arange(1000, 1000 + nh, dtype=np.int32)
    ent, sc, bh = oracle.entry_select(qemb, hemb, hg, hub_ids, Lh=nh, theta=-math.inf, med=7)
    cos = qemb.astype(np.float64) @ hemb.astype(np.float64).T
    assert (bh == np.argmax(cos, axis=1)).all()
    assert (ent == hub_ids[bh]).all()
    # score = 1 - d2/2 equals the cosine up to the FP32 rows' norm error (~1e-7)
    assert np.allclose(sc, cos.max(axis=1), rtol=0, atol=1e-6)
    ent2, _, _ = oracle.entry_select(qemb, hemb, hg, hub_ids, Lh=nh, theta=2.0, med=7)
    assert (ent2 == 7).all()


def test_hub_medoid_is_argmax_cosine_to_mean_direction():
    r = np.random.default_rng(6)
    hemb = _unit(r, 40, 8)
    m = hemb.astype(np.float64).sum(0)
    m /= np.linalg.norm(m)
    assert oracle.hub_medoid(hemb) == int(np.argmax(hemb.astype(np.float64) @ m))
