"""Pins for the oracle's graph-side functions: distances, exact kNN, alpha
pruning, medoid and connectivity repair.  Each test checks the oracle against
something other than itself: a closed form, an invariant, or an independent
brute force in exact arithmetic."""
from collections import deque
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2506_15986_amd import synth


def grid_data(n, d, seed, G=19, bound=16.0):
    r = np.random.default_rng(seed)
    x = r.normal(0, 3, size=(n, d))
    m = np.clip(np.rint(x * 2 ** G), -bound * 2 ** G, bound * 2 ** G - 1)
    return (m / 2 ** G).astype(np.float32)


# ---------------------------------------------------------------- distances
def test_sqdist_hand_value():
    assert oracle.sqdist([0, 0, 0], [3, 4, 0]) == 25.0
    assert oracle.sqdist([1.5, -2.0], [1.5, -2.0]) == 0.0


def test_sqdist_exact_on_grid_any_order():
    # On the dyadic grid every partial sum is exact, so a reversed-order sum
    # and an exact rational sum give the same bits.
    x = grid_data(50, 32, 1)
    for i in range(0, 50, 7):
        a, b = x[i], x[(i * 3 + 1) % 50]
        rev = 0.0
        for j in reversed(range(32)):
            t = float(a[j]) - float(b[j])
            rev += t * t
        exact = sum((Fraction(float(u)) - Fraction(float(v))) ** 2 for u, v in zip(a, b))
        assert oracle.sqdist(a, b) == rev == float(exact)


# ---------------------------------------------------------------- kNN
def test_knn_matches_exact_rational_bruteforce():
    base = grid_data(120, 8, 2)
    q = grid_data(6, 8, 3)
    ids, dd = oracle.knn(base, q, 10)
    for i in range(q.shape[0]):
        exact = [(sum((Fraction(float(u)) - Fraction(float(v))) ** 2
                      for u, v in zip(q[i], base[p])), p) for p in range(base.shape[0])]
        exact.sort()
        assert [p for _, p in exact[:10]] == ids[i].tolist()
        assert [float(v) for v, _ in exact[:10]] == dd[i].tolist()


def test_knn_ties_break_by_smaller_id_and_self_excluded():
    base = np.zeros((6, 2), np.float32)
    base[[1, 4]] = [1.0, 0.0]     # two points at distance 1 from the origin
    base[[2, 5]] = [0.0, 2.0]
    base[3] = [5.0, 5.0]
    ids, dd = oracle.knn(base, base[:1], 5)
    # ids 0 (itself, d=0), then 1,4 (d=1), then 2,5 (d=4)
    assert ids[0].tolist() == [0, 1, 4, 2, 5]
    ids, dd = oracle.knn(base, base, 3, exclude_self=True)
    assert ids[0].tolist() == [1, 4, 2]
    # 1 and 4 coincide: d2(1,4)=0, then origin 0 (d=1), then 2 vs 5 both d2=5
    assert ids[1].tolist() == [4, 0, 2]


# ---------------------------------------------------------------- alpha prune
def _line(n, seed):
    """n collinear points x = i (first coordinate), ids shuffled."""
    perm = np.random.default_rng(seed).permutation(n)
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)          # node perm[i] sits at coordinate i
    base = np.zeros((n, 4), np.float32)
    base[:, 0] = pos
    return base, pos


@pytest.mark.parametrize("alpha,expected", [
    (1.0, [1]),                       # MRNG: only the adjacent node per side
    (2.0, [1, 3, 7, 15]),             # "<=" keeps 2^t - 1 (a "<" rule would keep 1,2,4,8)
    (1.2, [1, 6]),                    # FP32 1.2 squared in FP64 is > 1.44: offset 6 survives
])
def test_alpha_prune_collinear_closed_form(alpha, expected):
    n = 30
    base, pos = _line(n, 5)
    cand, cd2 = oracle.knn(base, base, n - 1, exclude_self=True)
    g = oracle.alpha_prune(base, cand, cd2, R=n, alpha=alpha)
    node = int(np.where(pos == 15)[0][0])          # interior point at x = 15
    kept = [int(pos[c]) - 15 for c in g[node] if c >= 0]
    left = sorted(-o for o in kept if o < 0)
    right = sorted(o for o in kept if o > 0)
    exp_left = [m for m in expected if m <= 15]
    exp_right = [m for m in expected if m <= 14]
    assert left == exp_left and right == exp_right
    assert (g[:, -2:] == -1).all()


def test_alpha_exact_144_would_prune_offset_6():
    # a2 = 1.2f^2 is strictly above 1.44, which is why offset 6 survives;
    # with a2 == 1.44 exactly, 1.44 * 25 == 36 and "<=" would prune it.
    a2 = float(np.float32(1.2)) ** 2
    assert a2 * 25 > 36.0
    assert 1.44 * 25 <= 36.0 + 1e-12


def test_alpha_prune_properties_random():
    base = grid_data(400, 6, 7)
    K, R, alpha = 24, 10, 1.2
    cand, cd2 = oracle.knn(base, base, K, exclude_self=True)
    g = oracle.alpha_prune(base, cand, cd2, R, alpha)
    a2 = float(np.float32(alpha)) ** 2
    for p in range(0, 400, 13):
        kept = [c for c in g[p] if c >= 0]
        assert len(kept) == len(set(kept)) and p not in kept and len(kept) <= R - 2
        # kept list is a prefix-respecting subsequence of the candidates
        order = [int(c) for c in cand[p]]
        idx = [order.index(c) for c in kept]
        assert idx == sorted(idx)
        last = idx[-1]
        for t in range(last + 1):
            c = order[t]
            prev = [o for o in kept if order.index(o) < t]
            dom = any(a2 * oracle.sqdist(base[o], base[c]) <= cd2[p, t] for o in prev)
            assert dom == (c not in kept)


# ---------------------------------------------------------------- medoid
def test_medoid_symmetric_cross():
    d = 5
    pts = [np.zeros(d)]
    for j in range(d):
        for s in (1.0, -1.0):
            e = np.zeros(d)
            e[j] = s
            pts.append(e)
    base = np.array(pts, np.float32)
    perm = np.random.default_rng(0).permutation(len(base))
    shuffled = base[perm]
    assert oracle.medoid(shuffled) == int(np.where(perm == 0)[0][0])


def test_medoid_equals_exact_rational_argmin():
    for seed in range(3):
        base = grid_data(60, 6, 10 + seed)
        n = base.shape[0]
        mu = [sum(Fraction(float(base[i, j])) for i in range(n)) / n for j in range(6)]
        exact = min((sum((Fraction(float(base[i, j])) - mu[j]) ** 2 for j in range(6)), i)
                    for i in range(n))
        assert oracle.medoid(base) == exact[1]


# ---------------------------------------------------------------- repair
def _reach(graph, src, reverse=False):
    n = graph.shape[0]
    adj = [[] for _ in range(n)]
    for v in range(n):
        for w in graph[v]:
            if w >= 0:
                (adj[w] if reverse else adj[v]).append(v if reverse else w)
    seen = {src}
    dq = deque([src])
    while dq:
        v = dq.popleft()
        for w in adj[v]:
            if w not in seen:
                seen.add(w)
                dq.append(w)
    return seen


def test_repair_two_cycles_by_hand():
    # cluster A = {0,1,2} near the origin, cluster B = {3,4,5} near x = 100;
    # each cluster is a directed cycle in slot 0.  R = 4 (slots 2,3 for repair).
    base = np.array([[0, 0], [1, 0], [0, 1], [100, 0], [101, 0], [100, 1]], np.float32)
    g = -np.ones((6, 4), np.int32)
    g[0, 0], g[1, 0], g[2, 0] = 1, 2, 0
    g[3, 0], g[4, 0], g[5, 0] = 4, 5, 3
    rg, nf, nr = oracle.repair(base, g, 0)
    # forward: smallest unreached is 3; nearest reached node is 1 (d2 = 99^2)
    assert nf == 1 and rg[1, 2] == 3
    # reverse: 3 cannot reach 0; nearest node that can is 1 again
    assert nr == 1 and rg[3, 3] == 1
    assert _reach(rg, 0) == set(range(6)) and _reach(rg, 0, reverse=True) == set(range(6))
    # nothing else changed
    mask = np.ones_like(g, bool)
    mask[1, 2] = mask[3, 3] = False
    assert (rg[mask] == g[mask]).all()


def test_repair_listed_bridges_by_hand():
    # the two cycles above; 3's list names 2 (not its nearest reached node 1)
    # and 0, and 3's reverse bridge also comes from its list
    base = np.array([[0, 0], [1, 0], [0, 1], [100, 0], [101, 0], [100, 1]], np.float32)
    g = -np.ones((6, 4), np.int32)
    g[0, 0], g[1, 0], g[2, 0] = 1, 2, 0
    g[3, 0], g[4, 0], g[5, 0] = 4, 5, 3
    cand = -np.ones((6, 3), np.int32)
    cand[3] = [4, 2, 0]          # 4 is unreached: skipped; 2 is the first eligible
    rg, nf, nr = oracle.repair(base, g, 0, cand)
    assert nf == 1 and rg[2, 2] == 3 and rg[1, 2] == -1
    assert nr == 1 and rg[3, 3] == 2
    # an empty list falls back to the argmin
    rg2, _, _ = oracle.repair(base, g, 0, -np.ones((6, 3), np.int32))
    assert rg2[1, 2] == 3 and rg2[3, 3] == 1


def test_repair_from_global_lists_equals_argmin_rule():
    # with each point's exact global nearest neighbours as lists, the first
    # eligible entry is the argmin over all eligible points
    w = synth.scaled(synth.WORKLOADS["tiny"], n=1500)
    base = synth.base(w)
    cand, cd2 = oracle.knn(base, base, 64, exclude_self=True)
    g = oracle.alpha_prune(base, cand, cd2, 16, 1.2)
    m = oracle.medoid(base)
    a = oracle.repair(base, g, m)
    b = oracle.repair(base, g, m, cand)
    assert a[1] > 0 and a[2] > 0
    assert (a[0] == b[0]).all() and a[1:] == b[1:]


def test_build_graph_strongly_connected_tiny():
    w = synth.scaled(synth.WORKLOADS["tiny"], n=1500)
    base = synth.base(w)
    g, med, nf, nr, cand, _ = oracle.build_graph(base, knn_k=64, R=16, alpha=1.2)
    assert _reach(g, med) == set(range(1500))
    assert _reach(g, med, reverse=True) == set(range(1500))
    assert nf > 0        # the separated mixture needs forward bridges
    # pruned slots hold only candidates of the row, in candidate order
    for p in range(0, 1500, 37):
        kept = [c for c in g[p, :14] if c >= 0]
        order = cand[p].tolist()
        assert [order.index(c) for c in kept] == sorted(order.index(c) for c in kept)


# ---------------------------------------------------------------- grouped candidate lists
def test_knn_in_home_group_matches_masked_bruteforce():
    # independent brute force: the full exact distance matrix (rationals on
    # the grid are exact in FP64), a mask of the allowed pairs, a stable sort
    # by (d2, id)
    n, k = 90, 7
    base = grid_data(n, 6, 11)
    r = np.random.default_rng(5)
    groups = np.full((n, 3), -1, np.int32)
    groups[:, 0] = r.integers(0, 5, n)
    groups[:, 1] = r.integers(0, 5, n)            # sometimes a repeat of column 0
    groups[::4, 2] = r.integers(0, 5, (n + 3) // 4)
    groups[13] = [4, -1, -1]                      # no other column
    ids, dd = oracle.knn_in_home_group(base, groups, k)
    b = base.astype(np.float64)
    d2 = ((b[:, None, :] - b[None, :, :]) ** 2).sum(-1)
    for p in range(n):
        ok = [q for q in range(n) if q != p and groups[p, 0] in groups[q].tolist()]
        ok.sort(key=lambda q: (d2[p, q], q))
        want = ok[:k]
        assert ids[p, :len(want)].tolist() == want
        assert (ids[p, len(want):] == -1).all() and np.isinf(dd[p, len(want):]).all()
        assert dd[p, :len(want)].tolist() == [d2[p, q] for q in want]


def test_knn_in_home_group_one_group_is_plain_knn():
    base = grid_data(200, 8, 12)
    ids, dd = oracle.knn_in_home_group(base, np.zeros((200, 1), np.int32), 12)
    ref, rd = oracle.knn(base, base, 12, exclude_self=True)
    assert (ids == ref).all() and (dd == rd).all()


def test_knn_in_home_group_singleton_and_duplicates():
    # a group whose only member is its home point gets an empty list; exact
    # duplicates of the home point come first, by id, and the point itself
    # never appears
    base = np.zeros((5, 2), np.float32)
    base[3] = [3.0, 4.0]
    groups = np.array([[0], [0], [0], [1], [0]], np.int32)
    ids, dd = oracle.knn_in_home_group(base, groups, 3)
    assert ids[3].tolist() == [-1, -1, -1]
    assert ids[2].tolist() == [0, 1, 4] and dd[2].tolist() == [0.0, 0.0, 0.0]
    assert ids[0].tolist() == [1, 2, 4]


# ---------------------------------------------------------------- NSG-style candidates
def test_merge_candidates_by_hand():
    pool_ids = np.array([[0, 3, 5, -1], [2, 0, 1, 4]], np.int32)
    pool_d2 = np.array([[0.0, 2.0, 9.0, np.inf], [1.0, 3.0, 0.0, 3.0]])
    knn_ids = np.array([[3, 2], [0, 6]], np.int32)
    knn_d2 = np.array([[2.0, 5.0], [3.0, 7.0]])
    ids, dd = oracle.merge_candidates(pool_ids, pool_d2, knn_ids, knn_d2)
    # row 0: self (0) dropped, 3 once; row 1: self (1) dropped, ties by id
    assert ids[0].tolist() == [3, 2, 5, -1, -1, -1]
    assert dd[0, :3].tolist() == [2.0, 5.0, 9.0] and np.isinf(dd[0, 3:]).all()
    assert ids[1].tolist() == [2, 0, 4, 6, -1, -1]
    assert dd[1, :4].tolist() == [1.0, 3.0, 3.0, 7.0]


def test_nsg_graph_strongly_connected_and_sorted_rows():
    w = synth.scaled(synth.WORKLOADS["tiny"], n=1500)
    base = synth.base(w)
    g, med, nf, nr, cand, cd2 = oracle.build_graph_nsg(base, 64, 40, 16)
    assert _reach(g, med) == set(range(1500))
    assert _reach(g, med, reverse=True) == set(range(1500))
    # candidate rows: sorted by (d2, id), no self, no repeats
    for p in range(0, 1500, 53):
        row = [c for c in cand[p].tolist() if c >= 0]
        assert p not in row and len(set(row)) == len(row)
        keys = [(cd2[p, j], row[j]) for j in range(len(row))]
        assert keys == sorted(keys)
    # alpha = 1 keeps no more than alpha = 1.2 would from the same lists
    g12 = oracle.alpha_prune(base, cand, cd2, 16, 1.2)
    assert ((g[:, :14] >= 0).sum() <= (g12[:, :14] >= 0).sum())


def test_nsg_graph_two_clusters_on_a_line_by_hand():
    # ids 0..4 at x = 0..4 and ids 5..9 at x = 100..104.  knn_k = 2 keeps each
    # cluster to itself; the medoid (mean 52) ties between x = 4 and x = 100
    # and takes the smaller id, 4.  Searches from 4 over the kNN graph (width
    # 4) never leave the left cluster: for every right-hand point the pool is
    # [4, 3, 2, 1] (x = 0 is revealed last and rejected).  Merged with the kNN
    # list and pruned at alpha = 1 to R - 2 = 2, a line keeps the nearest point
    # on each side, so the left rows are path rows, while row 5 (x = 100)
    # keeps 6 and the search-built 4 (|x6 - x4| = 97 > |x5 - x4| = 96) and row
    # 9 (x = 104) loses 4 to 8 (99 <= 100).  Repair: 5..9 are unreached from 4;
    # 5's first reached candidate with a free slot R - 2 is 4 (one forward
    # bridge 4 -> 5); every node then reaches 4 through 5 -> 4 (no reverse
    # bridge).  The plain kNN + alpha = 1 graph instead needs a reverse bridge
    # 5 -> 4 in slot R - 1.
    base = np.zeros((10, 4), np.float32)
    base[:, 0] = [0, 1, 2, 3, 4, 100, 101, 102, 103, 104]
    g, med, nf, nr, cand, _ = oracle.build_graph_nsg(base, 2, 4, 4)
    want = [[1, -1, -1, -1], [0, 2, -1, -1], [1, 3, -1, -1], [2, 4, -1, -1], [3, -1, 5, -1],
            [6, 4, -1, -1], [5, 7, -1, -1], [6, 8, -1, -1], [7, 9, -1, -1], [8, -1, -1, -1]]
    assert med == 4 and (nf, nr) == (1, 0)
    assert g.tolist() == want
    assert cand[5].tolist()[:6] == [6, 7, 4, 3, 2, 1]
    gp, medp, nfp, nrp, _, _ = oracle.build_graph(base, 2, 4, 1.0)
    assert medp == 4 and (nfp, nrp) == (1, 1)
    assert gp[5].tolist() == [6, -1, -1, 4] and gp[4].tolist() == [3, -1, 5, -1]
