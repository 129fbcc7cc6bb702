"""GPU test of the continuous-batching server: each request's results are the
same alone and in the mix, and the mix really overlapped on the device."""
import numpy as np
import pytest
import torch

from paper_2506_15986_amd import synth
from tests.common import say, tiny_index

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("with_model", [True, False])
def test_results_same_alone_and_in_the_mix(with_model):
    from paper_2506_15986_amd import ann, serve
    from tests.test_gpu_driver import _model
    ix = tiny_index()
    w = synth.scaled(ix["w"], n_queries=3000)
    qs = synth.queries(w)
    base, g = _dev(ix["base"]), _dev(ix["graph"])
    model = _model(ix) if with_model else None
    kL = ((10, 32), (5, 16), (20, 48), (1, 1))
    # arrivals within microseconds: the queue outgrows the slots, so requests
    # wait and are admitted as slots free up
    sched = serve.poisson_schedule(qs, rate_per_s=1e7, sizes=(1, 120), kL=kL, seed=3)
    say("case: serve %d requests, model=%s" % (len(sched), with_model))
    srv = serve.Server(base, g, ix["medoid"], model=model, slots=3, slot_rows=200, k_max=20,
                       L_max=48)
    stats = srv.serve(sched)
    say("stats: %s" % stats)
    assert stats["requests"] == len(sched) and stats["queries"] == qs.shape[0]
    assert stats["max_slots_busy"] >= 2          # admitted while others were on the GPU
    assert stats["launches"] < len(sched)        # requests were packed together
    say("case: each request alone")
    plan = srv.plan
    for r in sched:
        q = _dev(r.queries)
        ent = ann.ann_entry_select(model, q)[0] if model is not None else None
        ids, dist, _, _ = ann.ann_search(base, g, q, ent, ix["medoid"], r.k, r.L, k_max=r.k,
                                         plan=plan)
        torch.cuda.synchronize()
        assert (ids.cpu().numpy() == r.ids).all(), r.rid
        assert (dist.cpu().numpy().view(np.uint32) == r.dist.view(np.uint32)).all(), r.rid


def test_rejects_requests_that_do_not_fit():
    from paper_2506_15986_amd import serve
    ix = tiny_index()
    srv = serve.Server(_dev(ix["base"]), _dev(ix["graph"]), ix["medoid"], slots=1, slot_rows=8,
                       k_max=10, L_max=32)
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, ix["q"][:9], 10, 32))
    with pytest.raises(ValueError):
        srv.submit(serve.Request(1, ix["q"][:2], 10, 64))
    with pytest.raises(ValueError):
        srv.submit(serve.Request(2, ix["q"][:2], 11, 10))


def test_admission_is_by_rows_of_the_pool():
    # a 64-row pool, launches of at most 40 rows and 4 streams: two 40-row
    # requests cannot share the pool, so they run one at a time although
    # streams are free; 16-row requests go two to a launch (32 rows) and two
    # launches fit in the pool at once; results equal the alone runs
    from paper_2506_15986_amd import ann, serve
    ix = tiny_index()
    w = synth.scaled(ix["w"], n_queries=640)
    qs = synth.queries(w)
    base, g = _dev(ix["base"]), _dev(ix["graph"])
    for b, most in ((40, 1), (16, 2)):
        sched = [serve.Request(i, qs[i * b:(i + 1) * b], 10, 32, 0.0) for i in range(640 // b)]
        srv = serve.Server(base, g, ix["medoid"], slots=4, slot_rows=40, pool_rows=64, k_max=10,
                           L_max=32)
        say("case: pool of 64 rows, launches of <= 40, requests of %d rows" % b)
        st = srv.serve(sched)
        say("stats: %s" % st)
        assert st["requests"] == len(sched)
        assert st["max_rows_in_use"] <= 64
        assert st["max_slots_busy"] == most
        for r in sched:
            ids, _, _, _ = ann.ann_search(base, g, _dev(r.queries), None, ix["medoid"], 10, 32,
                                          plan=srv.plan)
            assert (ids.cpu().numpy() == r.ids).all(), r.rid
