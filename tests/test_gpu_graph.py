"""GPU parity of the graph-construction entry points (exact kNN, medoid,
alpha pruning + repair) against the CPU oracle: bit-exact ids."""
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


def test_gt_knn_fp64_engine_tiny_exact():
    ix = tiny_index()
    say("case: gt_knn fp64 tiny")
    ids, dist = _ann().ann_gt_knn(_dev(ix["base"]), _dev(ix["q"]), 10)
    torch.cuda.synchronize()
    assert (ids.cpu().numpy() == ix["truth"]).all()
    assert (dist.cpu().numpy() == ix["truth_d2"].astype(np.float32)).all()


def test_gt_knn_int8_engine_exact():
    ix = int_index()
    say("case: gt_knn int8 20k")
    ids, dist = _ann().ann_gt_knn(_dev(ix["base"]), _dev(ix["q"]), 10)
    torch.cuda.synchronize()
    assert (ids.cpu().numpy() == ix["truth"]).all()
    assert (dist.cpu().numpy() == ix["truth_d2"].astype(np.float32)).all()


@pytest.mark.parametrize("n,nq,d,k,ints", [(1000, 77, 32, 13, False), (999, 65, 64, 130, True),
                                             (300, 1, 96, 300, False), (257, 200, 128, 5, True)])
def test_gt_knn_ragged_shapes(n, nq, d, k, ints):
    r = np.random.default_rng(n + nq)
    if ints:
        base = r.integers(0, 256, size=(n, d)).astype(np.float32)
        q = r.integers(0, 256, size=(nq, d)).astype(np.float32)
    else:
        base = (np.rint(r.normal(size=(n, d)) * 2 ** 12) / 2 ** 12).astype(np.float32)
        q = (np.rint(r.normal(size=(nq, d)) * 2 ** 12) / 2 ** 12).astype(np.float32)
    say("case: gt_knn n=%d nq=%d d=%d k=%d ints=%s" % (n, nq, d, k, ints))
    ids, dist = _ann().ann_gt_knn(_dev(base), _dev(q), k)
    torch.cuda.synchronize()
    ref_ids, ref_d2 = oracle.knn(base, q, k)
    assert (ids.cpu().numpy() == ref_ids).all()
    assert (dist.cpu().numpy()[ref_ids >= 0] == ref_d2[ref_ids >= 0].astype(np.float32)).all()


@pytest.mark.parametrize("n,nq,d,k,vmax", [
    (70_000, 300, 32, 10, 255),      # 17 column slices merged per row
    (20_000, 50, 256, 100, 255),     # widest rows, 4 slices
    (9_000, 700, 96, 300, 255),      # 2 slices of 301 kept entries
    (130, 600, 64, 200, 255),        # k above n: -1 padded
    (5_000, 3, 128, 1024, 255),      # largest k
    (20_000, 64, 160, 50, 3),        # values 0..3: long runs of equal distances
])
def test_int8_engine_slices_and_ties(n, nq, d, k, vmax):
    r = np.random.default_rng(n + d)
    base = r.integers(0, vmax + 1, size=(n, d)).astype(np.float32)
    q = r.integers(0, vmax + 1, size=(nq, d)).astype(np.float32)
    say("case: int8 kNN n=%d nq=%d d=%d k=%d values 0..%d" % (n, nq, d, k, vmax))
    ids, dist = _ann().ann_gt_knn(_dev(base), _dev(q), k)
    torch.cuda.synchronize()
    ref_ids, ref_d2 = oracle.knn(base, q, k)
    assert (ids.cpu().numpy() == ref_ids).all()
    ok = ref_ids >= 0
    assert (dist.cpu().numpy()[ok] == ref_d2[ok].astype(np.float32)).all()
    assert np.isinf(dist.cpu().numpy()[~ok]).all()


def test_int8_engine_exclude_self_with_duplicates():
    # rows repeated several times: the row's own column is dropped, its
    # duplicates stay (distance 0, by id)
    r = np.random.default_rng(11)
    base = r.integers(0, 256, size=(3000, 64)).astype(np.float32)
    base[1000:1040] = base[5]
    say("case: int8 kNN exclude_self with 41 copies of one row")
    ids, dist = _ann().ann_gt_knn(_dev(base), _dev(base), 60, exclude_self=True)
    torch.cuda.synchronize()
    ref_ids, ref_d2 = oracle.knn(base, base, 60, exclude_self=True)
    assert (ids.cpu().numpy() == ref_ids).all()
    assert (dist.cpu().numpy() == ref_d2.astype(np.float32)).all()


@pytest.mark.parametrize("n,d,k,vmax", [
    (70_000, 32, 20, 255),
    (70_000, 128, 128, 255),      # the graph build's shape: 128 dimensions, K = 128
    (66_000, 64, 30, 3),          # values 0..3: long runs of equal distances
])
def test_int8_all_pairs_in_cluster_order(n, d, k, vmax):
    # all pairs over one buffer of at least 65,536 rows run with rows and
    # columns grouped by their nearest sample row: every row's result equals
    # the pass in id order (a second buffer holding the same data) and, on a
    # sample of rows, the oracle's
    r = np.random.default_rng(n + d + vmax)
    base = r.integers(0, vmax + 1, size=(n, d)).astype(np.float32)
    base[500:530] = base[77]                     # duplicates of one row
    x = _dev(base)
    say("case: int8 all pairs in cluster order n=%d d=%d k=%d values 0..%d" % (n, d, k, vmax))
    ids, dist = _ann().ann_gt_knn(x, x, k, exclude_self=True)
    ids2, dist2 = _ann().ann_gt_knn(x, x.clone(), k, exclude_self=True)
    torch.cuda.synchronize()
    ids, dist, ids2, dist2 = ids.cpu().numpy(), dist.cpu().numpy(), ids2.cpu().numpy(), dist2.cpu().numpy()
    assert (ids == ids2).all()
    assert (dist.view(np.uint32) == dist2.view(np.uint32)).all()
    rows = np.concatenate([np.arange(0, n, n // 300), np.arange(500, 530), [77, n - 1]])
    ref_ids, ref_d2 = oracle.knn(base, base[rows], k + 1)
    for t, row in enumerate(rows):
        keep = [j for j in range(k + 1) if ref_ids[t, j] != row][:k]
        assert (ids[row] == ref_ids[t, keep]).all(), row
        assert (dist[row] == ref_d2[t, keep].astype(np.float32)).all(), row


def test_gt_knn_duplicates_tie_by_id_and_exclude_self():
    r = np.random.default_rng(3)
    base = r.integers(0, 4, size=(500, 32)).astype(np.float32)   # many exact ties
    base[100:110] = base[7]
    say("case: gt_knn ties")
    ids, dist = _ann().ann_gt_knn(_dev(base), _dev(base), 20, exclude_self=True)
    torch.cuda.synchronize()
    ref_ids, _ = oracle.knn(base, base, 20, exclude_self=True)
    assert (ids.cpu().numpy() == ref_ids).all()


def test_medoid_matches_oracle():
    ix = tiny_index()
    say("case: medoid")
    assert _ann().ann_medoid(_dev(ix["base"])) == ix["medoid"]
    ii = int_index()
    assert _ann().ann_medoid(_dev(ii["base"])) == ii["medoid"]


def test_build_graph_tiny_bit_exact():
    ix = tiny_index()
    say("case: build_graph tiny")
    g, med, (nf, nr) = _ann().ann_build_graph(_dev(ix["base"]), 64, 16, 1.2)
    torch.cuda.synchronize()
    assert med == ix["medoid"]
    assert (nf, nr) == (ix["nf"], ix["nr"])
    assert (g.cpu().numpy() == ix["graph"]).all()


def test_build_graph_int_bit_exact():
    ix = int_index()
    say("case: build_graph int 20k")
    g, med, (nf, nr) = _ann().ann_build_graph(_dev(ix["base"]), 64, 32, 1.2)
    torch.cuda.synchronize()
    assert med == ix["medoid"]
    assert (nf, nr) == (ix["nf"], ix["nr"])
    assert (g.cpu().numpy() == ix["graph"]).all()


def test_build_graph_small_alpha_variants():
    w = synth.scaled(synth.WORKLOADS["tiny"], n=1200)
    base = synth.base(w)
    for alpha, K, R in ((1.0, 24, 8), (2.0, 40, 12)):
        say("case: build_graph alpha=%.1f K=%d R=%d" % (alpha, K, R))
        ref, med, nf, nr, _, _ = oracle.build_graph(base, K, R, alpha)
        g, gm, (gf, gr) = _ann().ann_build_graph(_dev(base), K, R, alpha)
        torch.cuda.synchronize()
        assert gm == med and (gf, gr) == (nf, nr)
        assert (g.cpu().numpy() == ref).all()


def test_build_graph_partitioned_bit_exact():
    # candidates among the members of each point's home group (k-means
    # clusters, a second group for a third of the points, repeats, a home
    # group of one point, a small group), then prune / medoid / full-scan
    # repair; bit-exact against the oracle composition
    ann = _ann()
    ix = int_index()
    base = ix["base"]
    n = base.shape[0]
    K, R = 64, 32
    say("case: partitioned graph build, n=%d K=%d R=%d" % (n, K, R))
    km = oracle.kmeans_hubs(base, 4, 10, synth.kmeans_init(ix["w"], n, 4))
    groups = np.full((n, 2), -1, np.int32)
    groups[:, 0] = km["assign"]
    r = np.random.default_rng(3)
    sel = r.random(n) < 0.33
    groups[sel, 1] = r.integers(0, 4, int(sel.sum()))
    groups[7] = [4, -1]
    groups[100:110, 0] = 5
    groups[200:300, 1] = 5
    G = 6
    ref, med, nf, nr, _, _ = oracle.build_graph_grouped(base, groups, K, R, 1.2)
    g, m, br = ann.ann_build_graph_partitioned(_dev(base), K, R, 1.2, _dev(groups), G)
    torch.cuda.synchronize()
    assert m == med
    assert br == (nf, nr)
    assert (g.cpu().numpy() == ref).all()
    # the same build through the split entry points, a few groups per call
    say("case: group candidates in chunks + graph from candidates")
    bd, gd = _dev(base), _dev(groups)
    cand = torch.full((n, K), -7, dtype=torch.int32, device=bd.device)
    cd2 = torch.zeros((n, K), dtype=torch.float64, device=bd.device)
    for g0, g1 in ((0, 2), (2, 2), (2, 5), (5, 6)):
        ann.ann_group_candidates(bd, K, gd, G, g0, g1, cand, cd2)
    rc, rd = oracle.knn_in_home_group(base, groups, K)
    torch.cuda.synchronize()
    assert (cand.cpu().numpy() == rc).all()
    assert (cd2.cpu().numpy() == rd).all()
    g2, m2, br2 = ann.ann_graph_from_candidates(bd, cand, cd2, R, 1.2)
    torch.cuda.synchronize()
    assert m2 == med and br2 == (nf, nr)
    assert (g2.cpu().numpy() == ref).all()


def _merge_inputs(n, d, aw, bw, seed):
    r = np.random.default_rng(seed)
    base = (np.rint(r.normal(size=(n, d)) * 2 ** 10) / 2 ** 10).astype(np.float32)
    base[n // 2:n // 2 + 5] = base[3]            # equal distances, told apart by id
    a = r.integers(-1, n, size=(n, aw)).astype(np.int32)
    b = r.integers(-1, n, size=(n, bw)).astype(np.int32)
    if aw and bw:
        b[:, :min(aw, bw) // 2] = a[:, :min(aw, bw) // 2]   # repeats across the lists
    if aw:
        a[::7, 0] = np.arange(0, n, 7)                      # the row's own id
    return base, a, b


def _d2_rows(base, ids):
    # FP64 squared distances of row i to ids[i]; exact on this grid
    diff = base[np.maximum(ids, 0)].astype(np.float64) - base[:, None, :].astype(np.float64)
    return np.where(ids >= 0, (diff * diff).sum(-1), np.inf)


@pytest.mark.parametrize("n,d,aw,bw", [(300, 40, 37, 20), (129, 8, 0, 5), (200, 72, 300, 128),
                                       (64, 16, 900, 124), (97, 128, 1, 0)])
def test_merge_candidates_matches_oracle(n, d, aw, bw):
    say("case: merge_candidates n=%d d=%d aw=%d bw=%d" % (n, d, aw, bw))
    base, a, b = _merge_inputs(n, d, aw, bw, n + aw)
    ids, d2 = _ann().ann_merge_candidates(_dev(base), _dev(a) if aw else None,
                                          _dev(b) if bw else None)
    torch.cuda.synchronize()
    ea = a if aw else np.zeros((n, 0), np.int32)
    eb = b if bw else np.zeros((n, 0), np.int32)
    ref_ids, ref_d2 = oracle.merge_candidates(ea, _d2_rows(base, ea), eb, _d2_rows(base, eb))
    assert (ids.cpu().numpy() == ref_ids).all()
    assert (d2.cpu().numpy() == ref_d2).all()


def test_merge_candidates_rejects_ids_out_of_range():
    ann = _ann()
    base, a, b = _merge_inputs(100, 8, 10, 10, 5)
    a[17, 3] = 100
    say("case: merge_candidates id out of range")
    with pytest.raises(RuntimeError):
        ann.ann_merge_candidates(_dev(base), _dev(a), _dev(b))
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,d,knn_k,L,R,path", [(3000, 32, 32, 40, 16, 0),
                                                (2000, 64, 64, 100, 24, 0),
                                                (2500, 32, 16, 16, 24, 64)])
def test_nsg_graph_bit_exact(n, d, knn_k, L, R, path):
    from paper_2506_15986_amd import gate
    r = np.random.default_rng(n)
    if path:
        # uniform data: here the expanded nodes change about a fifth of the rows
        base = r.integers(0, 256, size=(n, d))
    else:
        cen = r.integers(30, 220, size=(12, d))
        base = np.clip(cen[r.integers(0, 12, n)] + r.integers(-25, 26, size=(n, d)), 0, 255)
    base = base.astype(np.float32)
    say("case: nsg graph n=%d d=%d knn_k=%d L=%d R=%d path=%d" % (n, d, knn_k, L, R, path))
    ix = gate.build_index_nsg(_dev(base), knn_k, R, L, path=path)
    g, m, nf, nr, _, _ = oracle.build_graph_nsg(base, knn_k, L, R, path=path)
    assert ix.medoid == m
    assert ix.bridges == (nf, nr)
    assert (ix.graph.cpu().numpy() == g).all()


def test_merge_candidates_single_point_and_self_only():
    base = np.array([[0.5, -1.0, 2.0, 0.25]], np.float32)
    a = np.array([[0, -1, 0]], np.int32)
    b = np.array([[-1, 0]], np.int32)
    say("case: merge_candidates n=1")
    ids, d2 = _ann().ann_merge_candidates(_dev(base), _dev(a), _dev(b))
    torch.cuda.synchronize()
    assert ids.cpu().numpy().tolist() == [[-1] * 5]
    assert np.isinf(d2.cpu().numpy()).all()
