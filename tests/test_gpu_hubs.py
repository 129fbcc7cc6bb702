"""GPU parity of hub selection (Lloyd k-means + Definition 3) and of the hub
topology features against the CPU oracle."""
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


@pytest.mark.parametrize("which,nh", [("tiny", 64), ("int", 64), ("tiny", 7)])
def test_select_hubs_bit_exact(which, nh):
    ix = tiny_index() if which == "tiny" else int_index()
    base = ix["base"]
    init = synth.kmeans_init(ix["w"], base.shape[0], nh)
    say("case: select_hubs %s nh=%d" % (which, nh))
    ref = oracle.kmeans_hubs(base, nh, 20, init)
    hub, cen, asg, steps = _ann().ann_select_hubs(_dev(base), nh, 20, _dev(init))
    torch.cuda.synchronize()
    assert steps == ref["steps"]
    assert (asg.cpu().numpy() == ref["assign"]).all()
    assert (cen.cpu().numpy() == ref["centroids"]).all()
    assert (hub.cpu().numpy() == ref["hub_ids"]).all()


@pytest.mark.parametrize("seed", [0, 2**63 + 11])
def test_select_hubs_from_a_seed_bit_exact(seed):
    # the library's seeded start (SplitMix64 + Floyd's sampling) is the
    # oracle's: the same centroids, assignment and hubs
    ix = int_index()
    base = ix["base"]
    nh = 48
    say("case: select_hubs from seed %d" % seed)
    init = oracle.hub_init_ids(base.shape[0], nh, seed)
    ref = oracle.kmeans_hubs(base, nh, 20, init)
    hub, cen, asg, steps = _ann().ann_select_hubs(_dev(base), nh, 20, seed=seed)
    torch.cuda.synchronize()
    assert steps == ref["steps"]
    assert (asg.cpu().numpy() == ref["assign"]).all()
    assert (cen.cpu().numpy() == ref["centroids"]).all()
    assert (hub.cpu().numpy() == ref["hub_ids"]).all()


@pytest.mark.parametrize("case", ["repeated", "wide", "odd_dim"])
def test_select_hubs_bit_exact_special_shapes(case):
    # repeated: 5 distinct rows behind 3,000 points and 64 centroids, so many
    # centroids coincide (exact ties, shortlists longer than their capacity:
    # the all-centroid fallback); wide: 960 dimensions (30 LDS stages per
    # pass) on the 2^-14 grid; odd_dim: 6 dimensions (no float4 rows: the
    # FP64 assignment kernel)
    r = np.random.default_rng(31)
    if case == "repeated":
        rows = r.integers(0, 256, size=(5, 64)).astype(np.float32)
        base = rows[r.integers(0, 5, size=3000)]
        nh = 64
    elif case == "wide":
        w = synth.scaled(synth.WORKLOADS["gist1m"], n=2000)
        base = synth.base(w)
        nh = 40
    else:
        base = (np.rint(r.normal(0, 4, size=(3000, 6)) * 2 ** 12) / 2 ** 12).astype(np.float32)
        nh = 24
    init = r.choice(base.shape[0], nh, replace=False).astype(np.int32)
    say("case: select_hubs %s" % case)
    ref = oracle.kmeans_hubs(base, nh, 20, init)
    hub, cen, asg, steps = _ann().ann_select_hubs(_dev(base), nh, 20, _dev(init))
    torch.cuda.synchronize()
    assert steps == ref["steps"]
    assert (asg.cpu().numpy() == ref["assign"]).all()
    assert (cen.cpu().numpy() == ref["centroids"]).all()
    assert (hub.cpu().numpy() == ref["hub_ids"]).all()


def test_select_hubs_empty_cluster():
    x = np.zeros((8, 4), np.float32)
    x[:, 0] = [0, 0, 10, 11, 0, 0, 10, 11]
    x[4:, 1] = 0.5
    init = np.array([0, 1, 2], np.int32)
    say("case: select_hubs empty cluster")
    ref = oracle.kmeans_hubs(x, 3, 5, init)
    hub, cen, asg, steps = _ann().ann_select_hubs(_dev(x), 3, 5, _dev(init))
    torch.cuda.synchronize()
    assert (asg.cpu().numpy() == ref["assign"]).all()
    assert (hub.cpu().numpy() == ref["hub_ids"]).all()


def test_hub_features_match_oracle():
    ix = tiny_index()
    base, g, med = ix["base"], ix["graph"], ix["medoid"]
    nh = 64
    init = synth.kmeans_init(ix["w"], base.shape[0], nh)
    km = oracle.kmeans_hubs(base, nh, 20, init)
    say("case: hub features tiny")
    ref, ref_ws = oracle.hub_features(base, g, med, km["hub_ids"], km["assign"], km["centroids"])
    raw, _ = oracle.hub_features(base, g, med, km["hub_ids"], km["assign"], km["centroids"],
                                 standardize=False)
    ann = _ann()
    args = (_dev(base), _dev(g), med, _dev(km["hub_ids"]), _dev(km["assign"]),
            _dev(km["centroids"]))
    f, wsz = ann.ann_hub_features(*args)
    fr, _ = ann.ann_hub_features(*args, standardise=False)
    torch.cuda.synchronize()
    assert (wsz.cpu().numpy() == ref_ws).all()
    assert np.allclose(fr.cpu().numpy(), raw, rtol=1e-5, atol=1e-6)
    assert np.allclose(f.cpu().numpy(), ref, rtol=0, atol=1e-4)


@pytest.mark.parametrize("which,k,levels,lam,iters", [
    ("int", 8, 2, 1.0, 5),       # integers 0..255, 64 clusters
    ("tiny", 4, 3, 0.5, 4),      # grid data, 64 clusters over 3 rounds
    ("tiny", 16, 1, 0.0, 6),     # no size term: Lloyd from spaced members
    ("int", 4, 2, 1e9, 2),       # a dominant size term: exact balance
])
def test_hbkm_hubs_bit_exact(which, k, levels, lam, iters):
    ann = _ann()
    ix = int_index() if which == "int" else tiny_index()
    base = ix["base"]
    say("case: HBKM %s k=%d levels=%d lambda=%g iters=%d" % (which, k, levels, lam, iters))
    hub, cen, asg = ann.ann_select_hubs_hbkm(_dev(base), k, levels, lam, iters)
    torch.cuda.synchronize()
    ref = oracle.hbkm_hubs(base, k, levels, lam, iters)
    assert (asg.cpu().numpy() == ref["assign"]).all()
    assert (cen.cpu().numpy() == ref["centroids"]).all()
    assert (hub.cpu().numpy() == ref["hub_ids"]).all()


def test_hbkm_more_clusters_than_distinct_points():
    # 64 clusters of 80 points with only 20 distinct rows: empty children and
    # the empty-cluster hub rule
    ann = _ann()
    r = np.random.default_rng(9)
    rows = r.integers(0, 256, size=(20, 32)).astype(np.float32)
    base = rows[r.integers(0, 20, size=80)]
    say("case: HBKM with repeated rows, 64 clusters")
    hub, cen, asg = ann.ann_select_hubs_hbkm(_dev(base), 8, 2, 0.0, 3)
    torch.cuda.synchronize()
    ref = oracle.hbkm_hubs(base, 8, 2, 0.0, 3)
    assert (asg.cpu().numpy() == ref["assign"]).all()
    assert (cen.cpu().numpy() == ref["centroids"]).all()
    assert (hub.cpu().numpy() == ref["hub_ids"]).all()
    assert len(set(hub.cpu().numpy().tolist())) == 64
