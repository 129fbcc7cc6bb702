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


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 8, 9, 17, 31])
def test_path_graph_ndc_closed_form_for_any_width(L):
    # path graph, query at base point j, entry i = j - D: the walk reaches j
    # after D + 1 expansions (D + 2 distances: the entry and its two sides,
    # then one new node per step); at j the pool holds the L nearest seen
    # nodes in the order j, j-1, j+1, j-2, j+2, ... (ties to the smaller id),
    # so node j+t is admitted (and expanded, revealing j+t+1) iff its rank 2t
    # is below L: floor((L-1)/2) extra expansions and as many extra distances
    # beyond j+1.  Holds while the entry's far side stays out of the pool
    # (L <= D + 1).
    n, i, j = 60, 10, 40
    D = j - i
    base, g = path_graph(n)
    r = oracle.search(base, g, base[j:j + 1], i, 1, L)
    assert r["ids"][0, 0] == j
    assert r["ndc"][0] == D + 3 + (L - 1) // 2
    assert r["hops"][0] == D + 1 + (L - 1) // 2


def _dead_end_graph():
    """Eight points on a line (x = position, other coordinates 0) and a
    directed graph with a dead end:
        id: 0  1   2  3   4  5  6  7
        x:  0  10  3  11  2  1  5  7
    E = 1 links to B = 2 and C = 3; B to E and D = 4; D back to B only; C to
    A = 0 and E; A to C and F = 5; F to A and G = 6; G to F and H = 7; H to
    G.  The query sits at x = 0, so the true nearest neighbour is A."""
    x = [0, 10, 3, 11, 2, 1, 5, 7]
    base = np.zeros((8, 4), np.float32)
    base[:, 0] = x
    g = np.array([[3, 5, -1], [2, 3, -1], [1, 4, -1], [0, 1, -1],
                  [2, -1, -1], [0, 6, -1], [5, 7, -1], [6, -1, -1]], np.int32)
    q = np.zeros((1, 4), np.float32)
    return base, g, q


def test_dead_end_graph_search_by_hand():
    # traced by hand from E (squared distances: A 0, F 1, D 4, B 9, G 25,
    # H 49, E 100, C 121):
    #  L=1: E -> pool [B] (C rejected) -> B reveals D -> D has nothing new:
    #       stuck at D, 4 distances, 3 expansions
    #  L=2: E -> [B, E]; C rejected (121 > 100); B reveals D -> [D, B]: stuck
    #  L=4: E -> [B, E, C]; B -> D; D; C reveals A; A reveals F; F reveals G
    #       (25 > 9, rejected): A found, 7 distances, expansions E B D C A F
    #  L=8: as L=4 but G and then H enter the pool: 8 distances, 8 expansions
    base, g, q = _dead_end_graph()
    want = {1: (4, 4, 3), 2: (4, 4, 3), 4: (0, 7, 6), 8: (0, 8, 8)}
    for L, (top, ndc, hops) in want.items():
        r = oracle.search(base, g, q, 1, 1, L, trace_cap=8)
        assert (r["ids"][0, 0], r["ndc"][0], r["hops"][0]) == (top, ndc, hops), L
    r = oracle.search(base, g, q, 1, 1, 4, trace_cap=8)
    assert r["trace"][0, :6].tolist() == [1, 2, 4, 3, 0, 5]


def test_labels_cost_is_taken_at_the_first_width_that_reaches():
    # from E (hub 0) the widths 1 and 2 do not reach A, 4 is the first that
    # does (7 distances) and 8 would cost 8; from F (hub 1) width 1 reaches A
    # at once: F reveals A (enters, 0 < 1) and G (25, rejected), A reveals C
    # (121, rejected): 4 distances.
    base, g, q = _dead_end_graph()
    truth = np.array([[0]], np.int32)
    hubs = np.array([1, 5, 4], np.int32)        # E, F, D
    lab, tab = oracle.make_labels(base, g, q, truth, np.array([[0, 1]], np.int32), hubs,
                                  [1, 2, 4, 8], 1)
    assert tab.tolist() == [[7, 4]] and lab.tolist() == [1]
    # widths 1 and 2 alone: E never reaches (-1); F still does
    lab, tab = oracle.make_labels(base, g, q, truth, np.array([[0, 1]], np.int32), hubs,
                                  [1, 2], 1)
    assert tab.tolist() == [[-1, 4]] and lab.tolist() == [1]
    # no candidate reaches: the label falls back to the first candidate
    lab, tab = oracle.make_labels(base, g, q, truth, np.array([[2, 0]], np.int32), hubs,
                                  [1, 2], 1)
    assert tab.tolist() == [[-1, -1]] and lab.tolist() == [2]
    # on the path graph every width reaches; the cost is the first width's
    # closed-form count (D + 3 + floor((L-1)/2)), not a later width's
    pb, pg = path_graph(60)
    lab, tab = oracle.make_labels(pb, pg, pb[40:41], np.array([[40]], np.int32),
                                  np.array([[0]], np.int32), np.array([10], np.int32), [3, 9], 1)
    assert tab.tolist() == [[30 + 3 + 1]]
    lab, tab = oracle.make_labels(pb, pg, pb[40:41], np.array([[40]], np.int32),
                                  np.array([[0]], np.int32), np.array([10], np.int32), [9, 3], 1)
    assert tab.tolist() == [[30 + 3 + 4]]


# ------------------------------------------- entry selection keyed by cosine
def _cosine_best_first(qe, he, hg, start, L):
    """Best-first search written directly on the high-tier graph's own key:
    (-cos(q, h), h), cos the FP64 dot product of the embeddings, from the
    hub `start`; the pool keeps the L best keys seen, each step expands the
    best unexpanded one.  Returns (best hub, its cos, distance count, hops)."""
    cos = lambda h: float(np.dot(qe.astype(np.float64), he[h].astype(np.float64)))  # noqa: E731
    pool = [(-cos(start), start, False)]
    seen = {start}
    ndc, hops = 1, 0
    while True:
        nxt = next((t for t, e in enumerate(pool) if not e[2]), None)
        if nxt is None:
            break
        key, h, _ = pool[nxt]
        pool[nxt] = (key, h, True)
        hops += 1
        for v in hg[h]:
            v = int(v)
            if v < 0 or v in seen:
                continue
            seen.add(v)
            ndc += 1
            kv = (-cos(v), v)
            if len(pool) < L or kv < pool[-1][:2]:
                pool.append((kv[0], v, False))
                pool.sort(key=lambda e: e[:2])
                del pool[L:]
    return pool[0][1], -pool[0][0], ndc, hops


def _cosine_top_s(he, s):
    """Row i: the s hubs j != i of largest (cos, -j)."""
    cos = he.astype(np.float64) @ he.astype(np.float64).T
    rows = []
    for i in range(he.shape[0]):
        order = sorted((j for j in range(he.shape[0]) if j != i), key=lambda j: (-cos[i, j], j))
        rows.append(order[:s])
    return np.array(rows, np.int32)


def test_entry_select_equals_cosine_keyed_search_on_exact_unit_vectors():
    # entries +-1/8 over 64 dimensions: every embedding has norm exactly 1
    # and every dot product is a multiple of 1/64, all exact in FP64, so
    # |a - b|^2 = 2 - 2 cos(a, b) holds exactly and the squared-L2 order is
    # the cosine order with ties (many, here) broken by the same index.  The
    # oracle's hub graph, hub entry and L2 search must then equal a search
    # keyed by cosine, step for step, at every width.
    r = np.random.default_rng(14)
    nh, e, nq, s = 96, 64, 40, 8
    he = (r.choice([-1.0, 1.0], size=(nh, e)) / 8).astype(np.float32)
    qe = (r.choice([-1.0, 1.0], size=(nq, e)) / 8).astype(np.float32)
    hg = oracle.hub_graph(he, s)
    assert (hg == _cosine_top_s(he, s)).all()
    mu = he.astype(np.float64).mean(0)
    start = int(np.argmax(he.astype(np.float64) @ mu))   # ties: numpy takes the first
    assert oracle.hub_medoid(he) == start
    hub_ids = np.arange(5000, 5000 + nh, dtype=np.int32)
    for Lh in (1, 4, 8, 16, nh):
        ent, sc, bh = oracle.entry_select(qe, he, hg, hub_ids, Lh, -math.inf, 3)
        r2 = oracle.search(he, hg, qe, start, 1, Lh)
        for i in range(nq):
            b, c, ndc, hops = _cosine_best_first(qe[i], he, hg, start, Lh)
            assert bh[i] == b and sc[i] == c, (Lh, i)
            assert (r2["ndc"][i], r2["hops"][i]) == (ndc, hops), (Lh, i)
        assert (ent == hub_ids[bh]).all()


def test_entry_select_matches_cosine_keyed_search_up_to_norm_error():
    # generic FP32 unit rows: their squared norms differ from 1 by ~1e-7, so
    # the L2 and cosine orders can only disagree between keys within that
    # error; every disagreement must be such a near tie
    r = np.random.default_rng(15)
    nh, e, nq, s = 128, 16, 60, 8
    he, qe = _unit(r, nh, e), _unit(r, nq, e)
    hg = oracle.hub_graph(he, s)
    cos = he.astype(np.float64) @ he.astype(np.float64).T
    ref = _cosine_top_s(he, s)
    for i in range(nh):
        for t in range(s):
            if hg[i, t] != ref[i, t]:
                assert abs(cos[i, hg[i, t]] - cos[i, ref[i, t]]) <= 1e-6
    start = oracle.hub_medoid(he)
    for Lh in (4, 12, 32):
        _, sc, bh = oracle.entry_select(qe, he, hg, np.arange(nh, dtype=np.int32), Lh,
                                        -math.inf, 0)
        qc = qe.astype(np.float64) @ he.astype(np.float64).T
        same = 0
        for i in range(nq):
            b, c, _, _ = _cosine_best_first(qe[i], he, hg, start, Lh)
            if bh[i] == b:
                same += 1
                assert abs(sc[i] - c) <= 1e-6
            else:
                assert abs(qc[i, bh[i]] - c) <= 1e-6, (Lh, i)
        assert same >= nq - 2
