"""GPU parity of ann_search (C-ABI) against the CPU oracle's beam search."""
import numpy as np
import pytest
import torch

import oracle
from tests.common import int_index, near_tie_certificate, say, tiny_index

pytestmark = pytest.mark.gpu


def _ann():
    from paper_2506_15986_amd import ann
    return ann


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _run(ix, entries, ks, Ls, plan, trace_cap=0, k_max=None):
    ann = _ann()
    base, g, q = _dev(ix["base"]), _dev(ix["graph"]), _dev(ix["q"])
    ent = _dev(np.asarray(entries, np.int32)) if entries is not None else None
    k = _dev(np.asarray(ks, np.int32))
    L = _dev(np.asarray(Ls, np.int32))
    ids, dist, st, tr = ann.ann_search(base, g, q, ent, ix["medoid"], k, L, k_max=k_max,
                                       plan=plan, trace_cap=trace_cap)
    torch.cuda.synchronize()
    out = dict(ids=ids.cpu().numpy(), dist=dist.cpu().numpy(), stats=st.cpu().numpy())
    if tr is not None:
        out["trace"] = tr.cpu().numpy()
    return out


def _plan(ix, L_max, **kw):
    ann = _ann()
    n, d = ix["base"].shape
    p = ann.default_plan(n, d, ix["graph"].shape[1], L_max)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("L", [10, 32, 100])
def test_fp64_mode_bitwise_on_tiny(L):
    ix = tiny_index()
    nq = ix["q"].shape[0]
    say("case: fp64 tiny L=%d nq=%d" % (L, nq))
    plan = _plan(ix, L, fp64=1)
    got = _run(ix, None, [10] * nq, [L] * nq, plan, trace_cap=2048)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L, trace_cap=2048)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["dist"] == ref["d2"].astype(np.float32)).all()
    assert (got["stats"][:, 0] == ref["ndc"]).all()
    assert (got["stats"][:, 1] == ref["ndc"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    assert (got["stats"][:, 3] == 0).all()
    assert (got["trace"] == ref["trace"]).all()


def test_fp32_mode_tiny_within_tolerance_and_certified():
    ix = tiny_index()
    nq, L = ix["q"].shape[0], 32
    say("case: fp32 tiny L=%d" % L)
    plan = _plan(ix, L)
    got = _run(ix, None, [10] * nq, [L] * nq, plan, trace_cap=2048)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L, trace_cap=2048)
    uncertified = 0
    for i in range(nq):
        if (got["trace"][i] == ref["trace"][i]).all():
            # same trajectory: same ids up to swaps of near-equal distances
            rd = ref["d2"][i]
            gd = got["dist"][i].astype(np.float64)
            assert np.all(np.abs(gd - rd) <= 1e-5 * np.maximum(rd, 1e-6))
            for t in range(10):
                if got["ids"][i, t] != ref["ids"][i, t]:
                    j = list(ref["ids"][i]).index(got["ids"][i, t]) if got["ids"][i, t] in ref["ids"][i] else -1
                    assert j >= 0 and abs(rd[j] - rd[t]) <= 1e-5 * rd[t]
        elif not near_tie_certificate(ix["base"], ix["graph"], ix["q"][i], ix["medoid"], L,
                                      got["trace"][i], ref["trace"][i]):
            uncertified += 1
    assert uncertified == 0


@pytest.mark.parametrize("L", [10, 64, 200])
def test_fp32_bitwise_on_integer_data(L):
    ix = int_index()
    nq = ix["q"].shape[0]
    say("case: fp32 int20k L=%d" % L)
    plan = _plan(ix, L)
    got = _run(ix, None, [10] * nq, [L] * nq, plan, trace_cap=4096)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L, trace_cap=4096)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["dist"] == ref["d2"].astype(np.float32)).all()
    assert (got["stats"][:, 1] == ref["ndc"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    assert (got["trace"] == ref["trace"]).all()


def test_uneven_k_L_and_entries():
    ix = int_index()
    nq = ix["q"].shape[0]
    r = np.random.default_rng(0)
    ks = r.choice([1, 5, 10, 37], size=nq)
    Ls = np.maximum(ks, r.choice([8, 40, 77, 129, 250], size=nq))
    ents = r.integers(0, ix["base"].shape[0], size=nq).astype(np.int32)
    say("case: uneven k/L with entries")
    plan = _plan(ix, 256)
    got = _run(ix, ents, ks, Ls, plan, k_max=40)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ents, ks, Ls, k_max=40)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["stats"][:, 1] == ref["ndc"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    assert np.isinf(got["dist"][ref["ids"] < 0]).all()


@pytest.mark.parametrize("filt", ["tag16", "tag12", "id32"])
def test_lossy_visited_table_keeps_results_exact(filt):
    # 10k ids need 313 bitset words; 2^8 slots forces a hash table, which
    # forgets ids: results, hops and the unique count stay exact
    ann = _ann()
    ix = int_index()
    nq, L = ix["q"].shape[0], 100
    say("case: lossy visited L=%d filter=%s" % (L, filt))
    kind = dict(tag16=ann.ANN_FILTER_TAG16, tag12=ann.ANN_FILTER_TAG12, id32=ann.ANN_FILTER_ID32)[filt]
    plan = _plan(ix, L, visited_log2=8, filter=kind)
    got = _run(ix, None, [10] * nq, [L] * nq, plan, trace_cap=4096)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L, trace_cap=4096)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    assert (got["trace"] == ref["trace"]).all()
    assert (got["stats"][:, 1] >= ref["ndc"]).all()
    over = got["stats"][:, 3] & 1
    assert over.any()
    # without overflow the unique count is exact
    ok = over == 0
    assert (got["stats"][ok, 0] == ref["ndc"][ok]).all()


def test_ragged_batches_and_invalid_rows():
    ix = int_index()
    base, g = ix["base"], ix["graph"]
    ann = _ann()
    for nq in (1, 3, 65):
        say("case: ragged nq=%d" % nq)
        q = ix["q"][:nq]
        sub = dict(ix, q=q)
        got = _run(sub, None, [10] * nq, [32] * nq, _plan(ix, 32))
        ref = oracle.search(base, g, q, ix["medoid"], 10, 32)
        assert (got["ids"] == ref["ids"]).all()
    # empty batch is a no-op
    say("case: nq=0")
    ids, dist, st, _ = ann.ann_search(_dev(base), _dev(g), _dev(ix["q"][:0]), None, ix["medoid"], 1, 1,
                                      k_max=1)
    torch.cuda.synchronize()
    assert ids.shape == (0, 1)
    # per-query invalid arguments: k > L, L > pool_cap, entry out of range
    say("case: invalid rows")
    q = ix["q"][:4]
    plan = _plan(ix, 64)
    got = _run(dict(ix, q=q), [0, 0, base.shape[0], 5], [10, 20, 5, 5], [5, 20, 10, 400], plan)
    assert (got["stats"][:, 3] == np.array([2, 0, 2, 2])).all()
    assert (got["ids"][[0, 2, 3]] == -1).all()
    assert (got["ids"][1] >= 0).all()


def test_k_equals_L_equals_1():
    ix = int_index()
    nq = ix["q"].shape[0]
    say("case: k=L=1")
    got = _run(ix, None, [1] * nq, [1] * nq, _plan(ix, 1))
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 1, 1)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()


def test_group16_and_multiwave_blocks_agree():
    ix = int_index()
    nq, L = ix["q"].shape[0], 64
    say("case: group16 / wpb=4")
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L)
    for kw in (dict(group=16), dict(waves_per_block=4), dict(waves_per_block=2, blocks=3)):
        got = _run(ix, None, [10] * nq, [L] * nq, _plan(ix, L, **kw))
        assert (got["ids"] == ref["ids"]).all(), kw
        assert (got["stats"][:, 1] == ref["ndc"]).all(), kw


@pytest.mark.parametrize("filt", ["bitset", "tag16", "tag12", "id32"])
def test_every_filter_form_matches_oracle_exactly_when_large(filt):
    # a table big enough never to forget: ids, hops and both counts exact
    ann = _ann()
    ix = int_index()
    nq, L = ix["q"].shape[0], 64
    kind = dict(bitset=ann.ANN_FILTER_BITSET, tag16=ann.ANN_FILTER_TAG16,
                tag12=ann.ANN_FILTER_TAG12, id32=ann.ANN_FILTER_ID32)[filt]
    say("case: filter=%s exact" % filt)
    plan = _plan(ix, L, visited_log2=14, filter=kind)
    got = _run(ix, None, [10] * nq, [L] * nq, plan, trace_cap=2048)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L, trace_cap=2048)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["trace"] == ref["trace"]).all()
    ok = (got["stats"][:, 3] & 1) == 0
    if filt == "bitset":
        assert ok.all()
    assert ok.mean() > 0.9
    assert (got["stats"][ok, 0] == ref["ndc"][ok]).all()
    assert (got["stats"][ok, 1] == ref["ndc"][ok]).all()


@pytest.mark.parametrize("W", [2, 4])
def test_several_waves_per_query_match(W):
    ann = _ann()
    ix = int_index()
    nq, L = ix["q"].shape[0], 64
    say("case: %d waves per query, integer data" % W)
    plan = _plan(ix, L, group=16, waves_per_query=W, waves_per_block=W)
    got = _run(ix, None, [10] * nq, [L] * nq, plan, trace_cap=2048)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, L, trace_cap=2048)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["trace"] == ref["trace"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    assert (got["stats"][:, 1] == ref["ndc"]).all()
    say("case: %d waves per query, uneven k, L and entries" % W)
    rng = np.random.default_rng(7)
    ks = rng.integers(1, 11, nq)
    Ls = rng.integers(10, 129, nq)
    ks = np.minimum(ks, Ls)
    ent = rng.integers(0, ix["base"].shape[0], nq)
    got = _run(ix, ent, ks, Ls, _plan(ix, 128, group=16, waves_per_query=W, waves_per_block=W),
               k_max=10)
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ent, ks, Ls, k_max=10)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    say("case: %d waves per query, lossy filter" % W)
    got = _run(ix, None, [10] * nq, [100] * nq,
               _plan(ix, 100, group=16, waves_per_query=W, waves_per_block=W, visited_log2=8))
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ix["medoid"], 10, 100)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    say("case: %d waves per query, ragged batches" % W)
    for m in (1, 3, 65):
        sub = dict(ix, q=ix["q"][:m])
        got = _run(sub, None, [10] * m, [32] * m,
                   _plan(ix, 32, group=16, waves_per_query=W, waves_per_block=W))
        ref = oracle.search(ix["base"], ix["graph"], ix["q"][:m], ix["medoid"], 10, 32)
        assert (got["ids"] == ref["ids"]).all(), m


@pytest.mark.parametrize("W", [2, 4])
def test_several_waves_per_query_equal_one_wave_on_float_data(W):
    ix = tiny_index()
    nq, L = ix["q"].shape[0], 48
    say("case: %d waves per query vs one, grid data" % W)
    one = _run(ix, None, [10] * nq, [L] * nq, _plan(ix, L, group=16), trace_cap=512)
    many = _run(ix, None, [10] * nq, [L] * nq,
                _plan(ix, L, group=16, waves_per_query=W, waves_per_block=W), trace_cap=512)
    assert (one["ids"] == many["ids"]).all()
    assert (one["dist"].view(np.uint32) == many["dist"].view(np.uint32)).all()
    assert (one["stats"] == many["stats"]).all()
    assert (one["trace"] == many["trace"]).all()


@pytest.mark.parametrize("d", [16, 32, 48, 64])
def test_group4_matches_oracle(d):
    # four lanes per vector (one quad), up to 64 dimensions: FP64 mode gives
    # the oracle's ids, distances, counts and expansion order bit for bit on
    # 16..64-dimensional integer data (d = 48 leaves the last chunk slot of
    # each lane empty)
    r = np.random.default_rng(d)
    n, nq, L = 3000, 64, 40
    base = r.integers(0, 256, size=(n, d)).astype(np.float32)
    q = r.integers(0, 256, size=(nq, d)).astype(np.float32)
    g, med, *_ = oracle.build_graph(base, knn_k=32, R=16, alpha=1.2)
    ix = dict(base=base, graph=g, q=q, medoid=med)
    say("case: group 4, d=%d" % d)
    ref = oracle.search(base, g, q, med, 10, L, trace_cap=256)
    for fp64 in (1, 0):
        got = _run(ix, None, [10] * nq, [L] * nq, _plan(ix, L, group=4, fp64=fp64), trace_cap=256)
        assert (got["ids"] == ref["ids"]).all(), fp64
        assert (got["stats"][:, 1] == ref["ndc"]).all(), fp64
        assert (got["stats"][:, 2] == ref["hops"]).all(), fp64
        assert (got["trace"] == ref["trace"]).all(), fp64
        assert (got["dist"] == ref["d2"].astype(np.float32)).all(), fp64


@pytest.mark.parametrize("L", [272, 330, 420, 512])
def test_pool_of_5_to_8_words_per_lane_matches_oracle(L):
    # pools of 257..512 entries are merged in place from 5..8 pool words per
    # lane (pool_cap = L rounded up to 16: 272, 336, 432, 512); integer data,
    # so FP32 distances are exact and everything must be the oracle's bits
    ix = int_index()
    nq = 24
    q = ix["q"][:nq]
    sub = dict(ix, q=q)
    plan = _plan(ix, L)
    assert 256 < plan.pool_cap <= 512
    say("case: L = %d (pool %d), k = 100" % (L, plan.pool_cap))
    ref = oracle.search(ix["base"], ix["graph"], q, ix["medoid"], 100, L, trace_cap=1024)
    got = _run(sub, None, [100] * nq, [L] * nq, plan, trace_cap=1024)
    assert (got["ids"] == ref["ids"]).all()
    assert (got["dist"] == ref["d2"].astype(np.float32)).all()
    assert (got["stats"][:, 2] == ref["hops"]).all()
    assert (got["trace"] == ref["trace"]).all()
    ok = (got["stats"][:, 3] & 1) == 0
    assert (got["stats"][ok, 0] == ref["ndc"][ok]).all()


def test_pool_wider_than_512_matches_oracle():
    # beam widths up to the 1024-entry pool (k = 100 at 10M points needs them)
    ix = int_index()
    nq = 24
    q = ix["q"][:nq]
    sub = dict(ix, q=q)
    say("case: L = 700 and 1024, k = 100")
    for L in (700, 1024):
        ref = oracle.search(ix["base"], ix["graph"], q, ix["medoid"], 100, L)
        got = _run(sub, None, [100] * nq, [L] * nq, _plan(ix, L))
        assert (got["ids"] == ref["ids"]).all(), L
        assert (got["stats"][:, 2] == ref["hops"]).all(), L
        assert (got["dist"] == ref["d2"].astype(np.float32)).all(), L


@pytest.mark.parametrize("wpq", [1, 2])
def test_results_do_not_depend_on_query_order(wpq):
    # the launch takes queries widest-expected-first (L x distance to the
    # entry); every query's ids, distances, counts and trace stay its own
    ix = int_index()
    nq = ix["q"].shape[0]
    r = np.random.default_rng(11)
    ent = r.integers(0, ix["base"].shape[0], nq).astype(np.int32)
    ks = r.integers(1, 11, nq).astype(np.int32)
    Ls = (ks + r.integers(0, 120, nq)).astype(np.int32)
    perm = r.permutation(nq)
    plan = _plan(ix, int(Ls.max()), group=16, waves_per_block=2 if wpq == 2 else 1,
                 waves_per_query=wpq)
    say("case: query order invariance wpq=%d" % wpq)
    a = _run(ix, ent, ks, Ls, plan, trace_cap=256, k_max=10)
    ixp = dict(ix, q=ix["q"][perm])
    b = _run(ixp, ent[perm], ks[perm], Ls[perm], plan, trace_cap=256, k_max=10)
    for key in ("ids", "dist", "stats", "trace"):
        assert (a[key][perm] == b[key]).all(), key
    plan.query_order = _ann().ANN_ORDER_AS_GIVEN          # no pre-pass: index order
    c = _run(ix, ent, ks, Ls, plan, trace_cap=256, k_max=10)
    for key in ("ids", "dist", "stats", "trace"):
        assert (a[key] == c[key]).all(), key
    ref = oracle.search(ix["base"], ix["graph"], ix["q"], ent, ks, Ls, k_max=10)
    assert (a["ids"] == ref["ids"]).all()
