"""Pins for the oracle's hub selection (Lloyd k-means + Definition 3) and the
two-tower model / InfoNCE / Adam (towers.py)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import towers
from paper_2506_15986_amd import synth


# ---------------------------------------------------------------- k-means hubs
def _mix(n=900, d=6, comps=5, seed=0, sep=40.0):
    r = np.random.default_rng(seed)
    mu = r.uniform(-sep, sep, size=(comps, d))
    lab = r.integers(0, comps, size=n)
    x = mu[lab] + r.normal(size=(n, d))
    m = np.rint(x * 2 ** 16)
    return (m / 2 ** 16).astype(np.float32), lab


def test_lloyd_objective_non_increasing():
    x, _ = _mix(seed=1, sep=3.0)
    init = np.random.default_rng(2).permutation(len(x))[:12].astype(np.int32)
    r = oracle.kmeans_hubs(x, 12, 30, init)
    obj = r["objective"]
    assert len(obj) >= 2
    assert all(b <= a * (1 + 1e-12) for a, b in zip(obj, obj[1:]))


def test_single_hub_is_medoid():
    x, _ = _mix(seed=3)
    r = oracle.kmeans_hubs(x, 1, 5, np.array([17], np.int32))
    assert r["hub_ids"][0] == oracle.medoid(x)


def test_every_point_its_own_hub():
    x, _ = _mix(n=50, seed=4)
    init = np.random.default_rng(5).permutation(50).astype(np.int32)
    r = oracle.kmeans_hubs(x, 50, 5, init)
    assert (r["hub_ids"] == init).all()


def test_matches_sklearn_lloyd():
    from sklearn.cluster import KMeans
    x, _ = _mix(n=600, seed=6, sep=4.0)
    nh, T = 8, 50
    init = np.random.default_rng(7).permutation(len(x))[:nh].astype(np.int32)
    r = oracle.kmeans_hubs(x, nh, T, init)
    km = KMeans(n_clusters=nh, init=x[init].astype(np.float64), n_init=1, max_iter=T,
                tol=0.0, algorithm="lloyd").fit(x.astype(np.float64))
    assert (km.labels_ == r["assign"]).mean() > 0.99
    # Definition 3: each hub is the member nearest its cluster mean
    for c in range(nh):
        mem = np.where(r["assign"] == c)[0]
        mu = x[mem].astype(np.float64).mean(0)
        dd = ((x[mem].astype(np.float64) - mu) ** 2).sum(1)
        assert r["hub_ids"][c] == mem[np.argmin(dd)]


def test_separated_mixture_one_seed_per_component_is_pure():
    x, lab = _mix(n=1000, comps=6, seed=8, sep=50.0)
    init = np.array([np.where(lab == c)[0][0] for c in range(6)], np.int32)
    r = oracle.kmeans_hubs(x, 6, 10, init)
    for c in range(6):
        assert len(set(lab[r["assign"] == c].tolist())) == 1
        assert lab[r["hub_ids"][c]] == c


def test_empty_cluster_gets_nearest_non_hub():
    # points 0 and 1 coincide and seed clusters 0 and 1; ties go to the lower
    # cluster index, so cluster 1 never gets a member
    x = np.array([[0, 0], [0, 0], [10, 0], [11, 0]], np.float32)
    r = oracle.kmeans_hubs(x, 3, 5, np.array([0, 1, 2], np.int32))
    assert r["assign"].tolist() == [0, 0, 2, 2]
    # cluster 0 = {0,1}: both at distance 0 from the mean, id 0 wins;
    # cluster 2 = {2,3}: both 0.5 from the mean, id 2 wins;
    # empty cluster 1 keeps centroid (0,0): nearest non-hub point is 1
    assert r["hub_ids"].tolist() == [0, 1, 2]


# ---------------------------------------------------------------- towers
def test_bf16_round_matches_torch_rne():
    r = np.random.default_rng(9)
    x = np.concatenate([r.normal(size=4000) * 10 ** r.uniform(-3, 3, size=4000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e-5]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    # torch rounds the float32 value; compare on inputs exact in float32
    x32 = x.astype(np.float32).astype(np.float64)
    assert (towers.bf16_round(x32) == ref).all()


def _params(r, din, h, e):
    return [r.uniform(-.3, .3, size=(h, din)), r.uniform(-.1, .1, size=h),
            r.uniform(-.3, .3, size=(e, h)), r.uniform(-.1, .1, size=e)]


def _loss(qp, hp, xq, xh, y, tau):
    eq, _ = towers.tower_forward(qp, xq, bf16=False)
    eh, _ = towers.tower_forward(hp, xh, bf16=False)
    return towers.infonce(eq, eh, y, tau)[0]


def test_gradients_match_finite_differences():
    r = np.random.default_rng(10)
    din, dh, h, e, B, nh, tau = 7, 9, 6, 5, 8, 11, 0.07
    qp, hp = _params(r, din, h, e), _params(r, dh, h, e)
    xq, xh = r.normal(size=(B, din)), r.normal(size=(nh, dh))
    y = r.integers(0, nh, size=B)
    loss, gq, gh, _, _ = towers.train_step_grads(qp, hp, xq, xh, y, tau, bf16=False)
    eps = 1e-6
    for params, grads in ((qp, gq), (hp, gh)):
        for P, G in zip(params, grads):
            flat = P.reshape(-1)
            gflat = np.asarray(G).reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + eps
                lp = _loss(qp, hp, xq, xh, y, tau)
                flat[idx] = old - eps
                lm = _loss(qp, hp, xq, xh, y, tau)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8


def test_gradients_match_torch_autograd_with_bf16_operands():
    # torch autograd through the same bf16-valued operands, with the rounding
    # of activations / gradients treated as identity in the backward pass
    r = np.random.default_rng(11)
    din, dh, h, e, B, nh, tau = 12, 15, 16, 8, 10, 13, 0.07
    qp, hp = _params(r, din, h, e), _params(r, dh, h, e)
    xq, xh = r.normal(size=(B, din)), r.normal(size=(nh, dh))
    y = r.integers(0, nh, size=B)
    loss, gq, gh, _, _ = towers.train_step_grads(qp, hp, xq, xh, y, tau, bf16=False)

    def tower(params, x):
        W1, b1, W2, b2 = params
        z = torch.relu(x @ W1.T + b1) @ W2.T + b2
        return z / z.norm(dim=1, keepdim=True)

    tq = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in qp]
    th = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in hp]
    eq = tower(tq, torch.tensor(xq))
    eh = tower(th, torch.tensor(xh))
    s = eq @ eh.T / tau
    L = torch.nn.functional.cross_entropy(s, torch.tensor(y))
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    for t, g in zip(tq + th, list(gq) + list(gh)):
        assert np.allclose(t.grad.numpy(), g, rtol=1e-10, atol=1e-12)


def test_infonce_closed_form_equal_hub_embeddings():
    r = np.random.default_rng(12)
    B, nh, e = 6, 1024, 8
    eq = r.normal(size=(B, e))
    eq /= np.linalg.norm(eq, axis=1, keepdims=True)
    one = r.normal(size=e)
    eh = np.tile(one / np.linalg.norm(one), (nh, 1))
    y = r.integers(0, nh, size=B)
    loss, deq, deh, ds = towers.infonce(eq, eh, y, 0.07)
    assert abs(loss - math.log(nh)) < 1e-12          # ln 1024 = 6.9315
    expect = np.full((B, nh), 1.0 / nh)
    expect[np.arange(B), y] -= 1.0
    assert np.allclose(ds, expect / B, atol=1e-15)


def test_adam_first_step_moves_by_lr_times_sign():
    r = np.random.default_rng(13)
    p = r.normal(size=20)
    g = r.normal(size=20)
    p1, m, v = towers.adam_update(p, g, np.zeros(20), np.zeros(20), 1, 1e-3)
    # bias-corrected m = g and v = g^2 after one step
    assert np.allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# ---------------------------------------------------------------- hub features
def _path(n):
    base = np.zeros((n, 4), np.float32)
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


def test_hub_features_path_graph_closed_form():
    # unit-spaced path: MinDeg 1, MaxDeg 2 -> x = 2 = deg, so the walk is a
    # BFS: 2 new nodes per depth 1..5, 9 expanded nodes x 2 sampled edges
    n = 40
    base, g = _path(n)
    assign = np.zeros(n, np.int32)
    hubs = np.array([20], np.int32)
    cen = base[hubs].astype(np.float64)
    f, ws = oracle.hub_features(base, g, 0, hubs, assign, cen, h=5, standardize=False)
    f = f[0]
    assert ws[0].tolist() == [1, 2, 2, 2, 2, 2]
    assert f[0] == 1.0                                 # out-degree 2 / R 2
    assert abs(f[1] - 2.0 / (2 * (n - 1) / n)) < 1e-12  # in-degree 2 / mean in-degree
    assert np.allclose(f[2:7], np.log2(3.0))
    assert abs(f[7] - np.log2(19.0)) < 1e-12
    assert np.allclose(f[8:12], [1, 1, 1, 0])          # nu = 1
    assert np.allclose(f[12:16], [3, 1, 5, np.sqrt(2.0)])
    assert abs(f[16] - 1.0) < 1e-12
    assert abs(f[18] - 20.0) < 1e-12                   # medoid at position 0
    assert f[19] == 0.0 and abs(f[20] - 1.0) < 1e-12
    assert abs(f[22] - 1.0) < 1e-12 and f[23] == 1.0
    assert (f[24:] == 0).all()


def test_hub_features_cluster_columns_on_a_two_cluster_path():
    # a 40-point path split into clusters 0..19 and 20..39, plus directed
    # edges 35 -> 16, 36 -> 16, 37 -> 16 in slot 2 (first slots keep their
    # path neighbour at distance 1, so nu = 1; MaxDeg 3, MinDeg 1 -> x = 2 on
    # the walk, whose nodes all have degree <= 2 there: the walk is the BFS
    # ball of depth 5).  mean in-degree = (78 + 3) / 40 = 2.025.
    #   hub 18 (cluster 0): walk 13..23; nodes 20..23 lie in cluster 1 -> col
    #     19 = 4 / 10; in-degrees 2 except node 16 (5) -> col 21 = (25 / 11)
    #     / 2.025; out-degrees all 2 -> col 20 = (22 / 11) / 3; centroid
    #     (9.5, 3) -> col 17 = sqrt(8.5^2 + 3^2)
    #   hub 30 (cluster 1): walk 25..35, all in cluster 1 -> col 19 = 0;
    #     in-degrees all 2 -> col 21 = 2 / 2.025; node 35 has out-degree 3 ->
    #     col 20 = (23 / 11) / 3; centroid (29.5, -4) -> col 17 = sqrt(16.25)
    n = 40
    base, g2 = _path(n)
    g = -np.ones((n, 3), np.int32)
    g[:, :2] = g2
    g[35:38, 2] = 16
    assign = (np.arange(n) >= 20).astype(np.int32)
    hubs = np.array([18, 30], np.int32)
    cen = np.zeros((2, 4))
    cen[0, :2] = [9.5, 3.0]
    cen[1, :2] = [29.5, -4.0]
    f, ws = oracle.hub_features(base, g, 0, hubs, assign, cen, h=5, standardize=False)
    assert ws.tolist() == [[1, 2, 2, 2, 2, 2]] * 2
    mean_in = 81.0 / 40.0
    assert abs(f[0, 17] - math.sqrt(8.5 ** 2 + 9.0)) < 1e-12
    assert abs(f[1, 17] - math.sqrt(16.25)) < 1e-12
    assert abs(f[0, 19] - 0.4) < 1e-15 and f[1, 19] == 0.0
    assert abs(f[0, 20] - 2.0 / 3.0) < 1e-12 and abs(f[1, 20] - 23.0 / 33.0) < 1e-12
    assert abs(f[0, 21] - (25.0 / 11.0) / mean_in) < 1e-12
    assert abs(f[1, 21] - 2.0 / mean_in) < 1e-12
    assert abs(f[0, 1] - 2.0 / mean_in) < 1e-12        # the hub's own in-degree
    assert abs(f[0, 16] - 20.0 / 20.0) < 1e-12          # cluster size / (n / n_hubs)


def test_hub_features_nearest_and_farthest_sampling():
    # node 0 at the origin links to 6 points at distances 1,2,3,4,5,6; every
    # other node has degree 1 -> MinDeg 1, MaxDeg 6, x(0) = max(2, 1) = 2:
    # one nearest (distance 1) and one farthest (distance 6) are sampled
    base = np.zeros((7, 4), np.float32)
    base[1:, 0] = [3, 1, 6, 2, 5, 4]
    g = -np.ones((7, 6), np.int32)
    g[0] = [1, 2, 3, 4, 5, 6]
    for v in range(1, 7):
        g[v, 0] = 0
    assign = np.zeros(7, np.int32)
    f, ws = oracle.hub_features(base, g, 0, np.array([0], np.int32), assign,
                                base[:1].astype(np.float64), h=1, standardize=False)
    assert ws[0].tolist() == [1, 2, 0, 0, 0, 0]
    assert abs(f[0, 7] - np.log2(3.0)) < 1e-12         # two sampled edges
    # walk nodes are ids 2 (distance 1) and 3 (distance 6); nu is the mean
    # distance to the first neighbour slot: (3 + 3+1+6+2+5+4) / 7
    nu = 24.0 / 7.0
    assert np.allclose(f[0, 12:16], np.array([3.5, 1.0, 6.0, 2.5]) / nu)
    assert abs(f[0, 22] - 3.5 / nu) < 1e-12


def test_hub_features_standardised_columns():
    base, g = _path(60)
    assign = (np.arange(60) // 20).astype(np.int32)
    hubs = np.array([10, 30, 50], np.int32)
    cen = np.stack([base[assign == c].astype(np.float64).mean(0) for c in range(3)])
    f, _ = oracle.hub_features(base, g, 30, hubs, assign, cen)
    assert np.allclose(f.mean(0), 0, atol=1e-12)
    sd = f.std(0)
    assert np.all((np.abs(sd - 1) < 1e-9) | (sd == 0))


# ---------------------------------------------------------------- HBKM (Algorithm 2)
def test_hbkm_one_pass_by_hand():
    # 1-D points 0, 1, 2, 10, 11, 12; k = 2, one level, one iteration,
    # lambda = 100.  Children start at members floor(1.5) = 1 (x = 1) and
    # floor(4.5) = 4 (x = 11); target m/k = 3; the penalty of child j is
    # lambda * (2 (s_j - 3) + 1) with s_j its size so far:
    #   x=0:  v = (1 - 500, 121 - 500)        -> 0, sizes (1, 0)
    #   x=1:  v = (0 - 300, 100 - 500)        -> 1, sizes (1, 1)
    #   x=2:  v = (1 - 300, 81 - 300)         -> 0, sizes (2, 1)
    #   x=10: v = (81 - 100, 1 - 300)         -> 1, sizes (2, 2)
    #   x=11: v = (100 - 100, 0 - 100)        -> 1, sizes (2, 3)
    #   x=12: v = (121 - 100, 1 + 100)        -> 0, sizes (3, 3)
    x = np.array([[0], [1], [2], [10], [11], [12]], np.float32)
    h = oracle.hbkm_hubs(x, 2, 1, 100.0, 1)
    assert h["assign"].tolist() == [0, 1, 0, 1, 1, 0]
    assert h["centroids"][:, 0].tolist() == [14.0 / 3.0, 22.0 / 3.0]
    # hubs: members nearest the means, (0, 2, 12) -> 2 and (1, 10, 11) -> 10
    assert h["hub_ids"].tolist() == [2, 3]      # ids of x = 2 and x = 10
    # without the penalty the two groups of the line separate
    h0 = oracle.hbkm_hubs(x, 2, 1, 0.0, 3)
    assert h0["assign"].tolist() == [0, 0, 0, 1, 1, 1]


def test_hbkm_without_penalty_is_lloyd():
    # lambda = 0, one level: the pass is the nearest-centroid assignment, so
    # the result is Lloyd's from the same starting members
    w = synth.scaled(synth.WORKLOADS["tiny"], n=3000)
    base = synth.base(w)
    k = 12
    init = np.array([(2 * j + 1) * 3000 // (2 * k) for j in range(k)], np.int32)
    ref = oracle.kmeans_hubs(base, k, 40, init)
    assert ref["steps"] < 40                     # Lloyd converged, so extra passes change nothing
    h = oracle.hbkm_hubs(base, k, 1, 0.0, 40)
    assert (h["assign"] == ref["assign"]).all()
    assert (h["centroids"] == ref["centroids"]).all()
    assert (h["hub_ids"] == ref["hub_ids"]).all()


def test_hbkm_dominant_penalty_balances_exactly_and_levels_nest():
    r = np.random.default_rng(4)
    base = (np.rint(r.normal(0, 3, size=(4096, 16)) * 2 ** 10) / 2 ** 10).astype(np.float32)
    # a penalty far above any distance: each point joins the smallest child
    h = oracle.hbkm_hubs(base, 4, 3, 1e9, 3)
    sizes = np.bincount(h["assign"], minlength=64)
    assert (sizes == 64).all()
    # a moderate penalty: level 2's clusters refine level 1's, and the hubs
    # are members of their clusters
    h2 = oracle.hbkm_hubs(base, 4, 2, 5.0, 4)
    h1 = oracle.hbkm_hubs(base, 4, 1, 5.0, 4)
    assert (h2["assign"] // 4 == h1["assign"]).all()
    assert (h2["assign"][h2["hub_ids"]] == np.arange(16)).all()
    # balance improves with the penalty
    s0 = np.bincount(oracle.hbkm_hubs(base, 4, 2, 0.0, 4)["assign"], minlength=16)
    s5 = np.bincount(h2["assign"], minlength=16)
    assert ((s5 - 256) ** 2).sum() < ((s0 - 256) ** 2).sum()


# ---------------------------------------------------------------- Definition 4 and Eq. 4
def test_hop_table_path_graph_and_unreachable():
    # directed path 0 -> 1 -> ... -> 9 and an isolated node 10
    g = -np.ones((11, 2), np.int32)
    for v in range(9):
        g[v, 0] = v + 1
    H = oracle.hop_table(g, np.array([0, 4], np.int32), np.array([0, 3, 9, 10], np.int32))
    assert H[:, 0].tolist() == [0, 3, 9, 255]
    assert H[:, 1].tolist() == [255, 255, 5, 255]       # edges only go forward


def test_hop_table_matches_library_shortest_paths():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    r = np.random.default_rng(7)
    n, R = 400, 3
    g = r.integers(-1, n, size=(n, R)).astype(np.int32)       # -1 = empty slot
    hubs = np.array([0, 17, 250, 399], np.int32)
    targets = r.integers(0, n, size=60).astype(np.int32)
    H = oracle.hop_table(g, hubs, targets)
    rows, cols = np.nonzero(g >= 0)
    A = csr_matrix((np.ones(len(rows)), (rows, g[rows, cols])), shape=(n, n))
    D = shortest_path(A, directed=True, unweighted=True, indices=hubs)
    want = np.where(np.isfinite(D[:, targets].T), D[:, targets].T, 255).astype(np.uint8)
    assert (H == want).all()


def test_sample_queues_by_definition():
    H = np.array([[2, 255], [3, 255], [5, 255], [20, 255], [255, 255]], np.uint8)
    pos, neg = oracle.sample_queues(H, 3, 15)
    assert pos[0].tolist() == [0, 1, 2] and neg[0].tolist() == [3, 4]   # m = 2
    assert pos[1].size == 0 and neg[1].size == 0                        # no query reaches hub 1


def test_hub_contrastive_closed_form_and_gradients():
    T = towers
    r = np.random.default_rng(3)
    P, N, tau = 3, 5, 0.1
    # all scores equal: L(V_i) = P log(P + N) for every hub
    eh = np.tile([[1.0, 0.0]], (2, 1))
    eq = np.tile([[1.0, 0.0]], (2 * (P + N), 1))
    loss, _, _ = T.hub_contrastive(eh, eq, P, N, tau)
    assert np.isclose(loss, P * np.log(P + N))
    # finite differences of the loss w.r.t. both embedding sets
    eh = r.normal(size=(2, 4))
    eq = r.normal(size=(2 * (P + N), 4))
    loss, deh, deq = T.hub_contrastive(eh, eq, P, N, tau)
    eps = 1e-6
    for (arr, grad) in ((eh, deh), (eq, deq)):
        for idx in [(0, 1), (1, 3), (arr.shape[0] - 1, 0)]:
            a2 = arr.copy()
            a2[idx] += eps
            lp = T.hub_contrastive(a2 if arr is eh else eh, a2 if arr is eq else eq, P, N, tau)[0]
            a2[idx] -= 2 * eps
            lm = T.hub_contrastive(a2 if arr is eh else eh, a2 if arr is eq else eq, P, N, tau)[0]
            assert np.isclose((lp - lm) / (2 * eps), grad[idx], rtol=1e-5, atol=1e-8)


# ---------------------------------------------------------------- Eq. 3 fusion
def _fusion_case(seed, nh=3, S=5, d=6, m=2, dk=3, dF=4):
    r = np.random.default_rng(seed)
    params = (r.normal(size=(m * dk, d)), r.normal(size=(m * dk, d)), r.normal(size=(m * dk, d)),
              r.normal(size=(dF, m * dk)))
    p = r.normal(size=(nh, d))
    U = r.normal(size=(nh, S, d))
    mask = np.ones((nh, S), np.uint8)
    mask[1, 3:] = 0
    mask[2, :] = 0                                 # a hub without tokens
    return params, p, U, mask, m


def test_fusion_single_token_is_linear_and_no_token_is_zero():
    # one present token: every softmax is 1, so F = (U_0 WV^T) WO^T
    params, p, U, mask, m = _fusion_case(1)
    mask[:] = 0
    mask[0, 2] = 1
    F, _ = towers.fusion_forward(params, p, U, mask, m)
    WQ, WK, WV, WO = params
    assert np.allclose(F[0], (U[0, 2] @ WV.T) @ WO.T)
    assert (F[1] == 0).all() and (F[2] == 0).all()


def test_fusion_matches_per_head_softmax_by_hand():
    params, p, U, mask, m = _fusion_case(2)
    F, _ = towers.fusion_forward(params, p, U, mask, m)
    WQ, WK, WV, WO = params
    dk = WQ.shape[0] // m
    i = 1                                          # tokens 0..2 present
    heads = []
    for j in range(m):
        sl = slice(j * dk, (j + 1) * dk)
        sc = np.array([(p[i] @ WQ[sl].T) @ (U[i, s] @ WK[sl].T) for s in range(3)]) / np.sqrt(dk)
        w = np.exp(sc) / np.exp(sc).sum()
        heads.append(sum(w[s] * (U[i, s] @ WV[sl].T) for s in range(3)))
    assert np.allclose(F[i], np.concatenate(heads) @ WO.T)


def test_fusion_gradients_match_finite_differences():
    params, p, U, mask, m = _fusion_case(3)
    r = np.random.default_rng(4)
    dF = r.normal(size=(3, 4))
    F, cache = towers.fusion_forward(params, p, U, mask, m)
    grads = towers.fusion_backward(cache, dF)
    eps = 1e-6
    for w_i in range(4):
        for idx in [(0, 0), (1, 2), (params[w_i].shape[0] - 1, params[w_i].shape[1] - 1)]:
            pp = [np.array(x, np.float64) for x in params]
            pp[w_i][idx] += eps
            lp = (towers.fusion_forward(pp, p, U, mask, m)[0] * dF).sum()
            pp[w_i][idx] -= 2 * eps
            lm = (towers.fusion_forward(pp, p, U, mask, m)[0] * dF).sum()
            assert np.isclose((lp - lm) / (2 * eps), grads[w_i][idx], rtol=1e-5, atol=1e-8)


def test_tower_input_gradient_matches_finite_differences():
    r = np.random.default_rng(5)
    params = (r.normal(size=(7, 5)) * 0.5, r.normal(size=7), r.normal(size=(4, 7)) * 0.5, r.normal(size=4))
    x = r.normal(size=(3, 5))
    de = r.normal(size=(3, 4))
    e, cache = towers.tower_forward(params, x, bf16=False, in_scale=0.5)
    dx = towers.tower_backward_input(cache, de, bf16=False, in_scale=0.5)
    eps = 1e-6
    for idx in [(0, 0), (1, 3), (2, 4)]:
        x2 = x.copy()
        x2[idx] += eps
        lp = (towers.tower_forward(params, x2, bf16=False, in_scale=0.5)[0] * de).sum()
        x2[idx] -= 2 * eps
        lm = (towers.tower_forward(params, x2, bf16=False, in_scale=0.5)[0] * de).sum()
        assert np.isclose((lp - lm) / (2 * eps), dx[idx], rtol=1e-5, atol=1e-8)


def test_sample_queues_hand_table():
    # hub 0: hops (2, 5, 255, 3, 20) -> m = 2; t_pos 1: positives H <= 3 ->
    # queries 0, 3; t_neg 10: negatives H >= 12 or unreachable -> 2, 4.
    # hub 1 reaches no query: neither queue.  hub 2: all at 0 -> all positive
    H = np.array([[2, 255, 0], [5, 255, 0], [255, 255, 0], [3, 255, 0], [20, 255, 0]], np.uint8)
    pos, neg = oracle.sample_queues(H, 1, 10)
    assert [p.tolist() for p in pos] == [[0, 3], [], [0, 1, 2, 3, 4]]
    assert [n.tolist() for n in neg] == [[2, 4], [], []]


def test_splitmix64_published_outputs():
    # the generator's commonly printed check values: five outputs from state
    # 1234567
    assert oracle.splitmix64(1234567, 5) == [6457827717110365317, 3203168211198807973,
                                             9817491932198370423, 4593380528125082431,
                                             16408922859458223821]
    # outputs are the finaliser of seed + i * increment: a run from a later
    # state continues the sequence
    xs = oracle.splitmix64(99, 6)
    assert oracle.splitmix64(99 + 3 * 0x9E3779B97F4A7C15, 3) == xs[3:]


def test_floyd_sample_is_uniform_over_subsets():
    # every sequence of draws for n = 6, m = 3 (t in 0..3, 0..4, 0..5: 120
    # sequences) gives 3 distinct values, and each of the 20 subsets comes
    # from exactly 6 of them
    import itertools
    counts = {}
    for ts in itertools.product(range(4), range(5), range(6)):
        it = iter(ts)
        v = oracle.floyd_sample(6, 3, lambda j: next(it))
        assert len(set(v)) == 3 and all(0 <= x < 6 for x in v)
        counts[frozenset(v)] = counts.get(frozenset(v), 0) + 1
    assert len(counts) == 20 and set(counts.values()) == {6}


def test_hub_init_ids_ranges_and_special_cases():
    # m = n takes every id, in order (each later j is taken or its t is)
    assert (oracle.hub_init_ids(10, 10, 3) == np.arange(10)).all()
    for n, m, seed in ((7, 1, 1), (1000, 64, 0), (10**7, 1024, 2**64 - 1)):
        v = oracle.hub_init_ids(n, m, seed)
        assert len(v) == m and len(set(v.tolist())) == m and v.min() >= 0 and v.max() < n
    # the draw from 0..j maps the largest 64-bit output to j and 0 to 0
    assert ((2**64 - 1) * 1000) >> 64 == 999 and (0 * 1000) >> 64 == 0
    # one id out of n: the first output's top bits, x * n / 2^64
    x0 = oracle.splitmix64(5, 1)[0]
    assert oracle.hub_init_ids(1000, 1, 5)[0] == x0 * 1000 // 2**64
