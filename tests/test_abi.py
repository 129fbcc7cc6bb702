"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments on the host before touching the device (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ann.h")
LIB = os.path.join(ROOT, "paper_2506_15986_amd", "libann.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ann_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libann.so not built")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "ann_search" in names and "ann_last_error" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2506_15986_amd import ann
    for n in declared_functions():
        if n in ("ann_last_error", "ann_version", "ann_workspace_size", "ann_default_plan"):
            continue
        assert hasattr(ann, n), n


def test_search_rejects_bad_arguments_before_any_device_work(lib):
    from paper_2506_15986_amd import ann
    lib = ann._lib
    fake = ctypes.c_void_p(0x10000)      # never dereferenced: validation fails first
    odd = ctypes.c_void_p(0x10004)       # not 16-byte aligned

    wsb = ann.workspace_size("search", 1000, 32, 4)    # counter, query order and its keys

    def call(**kw):
        a = dict(base=fake, n=1000, dim=32, graph=fake, R=16, queries=fake, nq=4, entry=None,
                 medoid=0, k=fake, L=fake, k_max=10, ids=fake, dist=fake, stats=None, trace=None,
                 trace_cap=0, plan=None, ws=fake, wsb=wsb, stream=None)
        a.update(kw)
        return lib.ann_search(a["base"], a["n"], a["dim"], a["graph"], a["R"], a["queries"],
                              a["nq"], a["entry"], a["medoid"], a["k"], a["L"], a["k_max"],
                              a["ids"], a["dist"], a["stats"], a["trace"], a["trace_cap"],
                              a["plan"], a["ws"], a["wsb"], a["stream"])

    assert call(base=None) == ann.ANN_EINVAL
    assert "NULL" in ann.last_error()
    assert call(n=0) == ann.ANN_EINVAL
    assert call(dim=30) == ann.ANN_ENOTSUP
    assert call(dim=2048) == ann.ANN_ENOTSUP
    assert call(R=65) == ann.ANN_ENOTSUP
    assert call(R=0) == ann.ANN_EINVAL
    assert call(medoid=1000) == ann.ANN_EINVAL
    assert call(base=odd) == ann.ANN_EINVAL
    assert call(wsb=16) == ann.ANN_EINVAL
    assert call(wsb=wsb - 1) == ann.ANN_EINVAL
    assert call(k_max=0) == ann.ANN_EINVAL
    bad = ann.ann_search_plan(pool_cap=1040, visited_log2=12, group=8, waves_per_block=1,
                              blocks=0, fp64=0)
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    bad.pool_cap, bad.group = 64, 12
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    bad.group, bad.waves_per_query, bad.waves_per_block = 8, 3, 1
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    bad.waves_per_query = 2                      # needs waves_per_block == 2
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    bad.waves_per_block = 2                      # group 8 cannot share a query
    assert call(plan=ctypes.byref(bad)) == ann.ANN_ENOTSUP
    bad.waves_per_query, bad.waves_per_block, bad.group = 1, 1, 4
    assert call(plan=ctypes.byref(bad), dim=68) == ann.ANN_ENOTSUP   # group 4: dim <= 64
    bad.group = 8
    assert call(plan=ctypes.byref(bad), dim=132) == ann.ANN_ENOTSUP  # group 8: dim <= 128
    bad.group = 12
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    bad.group, bad.query_order = 8, 2
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    # nq == 0 is valid and enqueues nothing
    assert call(nq=0) == ann.ANN_OK


def test_default_plan_and_workspace():
    from paper_2506_15986_amd import ann
    p = ann.default_plan(1_000_000, 128, 32, 200)
    assert p.pool_cap == 208 and p.group == 8 and p.fp64 == 0 and p.filter == ann.ANN_FILTER_AUTO
    p = ann.default_plan(1_000_000, 960, 64, 400)
    assert p.pool_cap == 400 and p.group == 16
    assert ann.default_plan(10, 32, 16, 1).pool_cap == 16
    assert ann.default_plan(10, 32, 16, 600).pool_cap == 608
    with pytest.raises(ann.AnnError):
        ann.default_plan(10, 32, 16, 1025)
    assert ann.workspace_size("search", 1000, 32, 1) == 256
    assert ann.workspace_size("search", 1000, 32, 10) >= 256 + 2 * 40
    assert ann.workspace_size("search", 1000, 32, 100000) >= 256 + 2 * 400000


def test_kernel_names_unique_across_translation_units():
    # each .hip file is its own code object inside libann.so; two code objects
    # exporting the same kernel symbol must not happen
    src = os.path.join(ROOT, "paper_2506_15986_amd", "csrc")
    seen = {}
    for f in sorted(os.listdir(src)):
        if not f.endswith(".hip"):
            continue
        text = open(os.path.join(src, f)).read()
        for name in re.findall(r"__global__\s+void\s+(?:__launch_bounds__\([^)]*\)\s+)?(\w+)\s*\(", text):
            assert name not in seen, "kernel %s defined in %s and %s" % (name, seen[name], f)
            seen[name] = f
    assert len(seen) > 20


def _lds(pool_cap, filter_words, fp64=False, dim=128):
    # FP32 pools of up to 512 entries are merged in place (one buffer), the
    # others in two ping-pong buffers
    ks = 8 if fp64 else 4
    bufs = 1 if (not fp64 and pool_cap <= 512) else 2
    b = (dim * 4 + 15) // 16 * 16 + bufs * pool_cap * ks + 64 * ks + bufs * pool_cap * 4 + \
        64 * 4 + 64 + filter_words * 4
    return (b + 15) // 16 * 16


def test_plan_lds_and_filter_forms():
    from paper_2506_15986_amd import ann
    P = lambda **kw: ann.make_plan(**dict(dict(pool_cap=64, visited_log2=12, group=8,
                                               waves_per_block=1, blocks=0, fp64=0,
                                               filter=ann.ANN_FILTER_AUTO), **kw))
    lds = lambda p, n: ann.ann_search_plan_lds(p, n, 128)
    # 10k ids: 313 bitset words fit in the 2048-word tag table -> bitset
    assert lds(P(), 10_000) == _lds(64, 313)
    # 1M ids: 31,250 bitset words do not -> 10-bit tags in 12-bit ways, five
    # to a 64-bit set, in the bytes of 16-bit tags at 2 bytes per slot
    assert lds(P(), 1_000_000) == _lds(64, 2048)
    assert lds(P(filter=ann.ANN_FILTER_TAG12), 1_000_000) == _lds(64, 2048)
    assert lds(P(filter=ann.ANN_FILTER_TAG16), 1_000_000) == _lds(64, 2048)
    # 12-bit ways hold tags of at most 11 bits: 2^21 ids with 2^10 sets fit,
    # 2^22 do not (AUTO then takes 16-bit tags, same bytes)
    assert lds(P(filter=ann.ANN_FILTER_TAG12), 1 << 21) == _lds(64, 2048)
    assert lds(P(filter=ann.ANN_FILTER_TAG12), 1 << 22) == 0
    assert lds(P(), 1 << 22) == _lds(64, 2048)
    assert lds(P(visited_log2=10), 1_000_000) == _lds(64, 512)
    assert lds(P(filter=ann.ANN_FILTER_ID32), 1_000_000) == _lds(64, 4096)
    assert lds(P(filter=ann.ANN_FILTER_BITSET), 1_000_000) == 0        # cannot hold 1M bits
    assert lds(P(filter=ann.ANN_FILTER_BITSET, visited_log2=14), 500_000) == _lds(64, 15625)
    # tags of 2^30 ids with 2^10 sets need 20 bits: AUTO takes 32-bit ids
    assert lds(P(), 1 << 30) == _lds(64, 4096)
    assert lds(P(filter=ann.ANN_FILTER_TAG16), 1 << 30) == 0
    # 2^25 ids with 2^10 sets: 15-bit tags still fit
    assert lds(P(), 1 << 25) == _lds(64, 2048)
    assert lds(P(fp64=1), 10_000) == _lds(64, 313, fp64=True)
    # in place up to 512 entries, two buffers beyond
    assert lds(P(pool_cap=256), 10_000) == _lds(256, 313)
    assert lds(P(pool_cap=272), 10_000) == _lds(272, 313)
    assert lds(P(pool_cap=512), 10_000) == _lds(512, 313)
    assert lds(P(pool_cap=528), 10_000) == _lds(528, 313)
    assert _lds(528, 313) - _lds(512, 313) > 512 * 8
    assert _lds(272, 313) - _lds(256, 313) == 16 * 8
    # FP64 keys always take two buffers
    assert lds(P(pool_cap=256, fp64=1), 10_000) == _lds(256, 313, fp64=True)
    assert lds(P(filter=7), 10_000) == 0                                  # invalid form
    assert lds(P(filter=5), 10_000) == 0


def test_autotune_candidates():
    from paper_2506_15986_amd import ann
    c = ann.ann_autotune_candidates(1_000_000, 128, 32, 160)
    d = ann.default_plan(1_000_000, 128, 32, 160)
    assert c[0].as_dict() == d.as_dict() and d.waves_per_query == 1
    # 2 groups x 4 filter sizes x 3 workgroup sizes, plus group 16 x 4 sizes x
    # 2 and 4 waves per query
    assert len(c) == 24 + 8
    assert len({tuple(p.as_dict().items()) for p in c}) == 32
    assert all(p.pool_cap == 160 and p.blocks == 0 and p.fp64 == 0 for p in c)
    assert {p.group for p in c} == {8, 16} and {p.visited_log2 for p in c} == {10, 11, 12, 13}
    mw = [p for p in c if p.waves_per_query > 1]
    assert len(mw) == 8 and all(p.group == 16 and p.waves_per_block == p.waves_per_query
                                for p in mw)
    # wide vectors: group 16 only
    c = ann.ann_autotune_candidates(1_000_000, 960, 64, 100)
    assert len(c) == 12 + 8 and {p.group for p in c} == {16}
    assert ann.ann_autotune_candidates(10, 32, 16, 1025) == []


def test_batch_driver_rejects_bad_arguments_without_gpu_work():
    from paper_2506_15986_amd import ann
    assert ann._lib.ann_query_run(None, 3, None) == ann.ANN_EINVAL
    b = ann.ann_query_batch()
    assert ann._lib.ann_query_run(ctypes.byref(b), 0, None) == ann.ANN_EINVAL
    assert ann._lib.ann_query_run(ctypes.byref(b), 2, None) == ann.ANN_EINVAL     # null base
    h = ctypes.c_void_p()
    assert ann._lib.ann_query_graph_create(ctypes.byref(b), 4, ctypes.byref(h)) == ann.ANN_EINVAL
    assert not h.value
    assert ann._lib.ann_query_graph_launch(None, None) == ann.ANN_EINVAL
    ann._lib.ann_query_graph_destroy(None)
    best = ann.ann_search_plan()
    assert ann._lib.ann_autotune_search(None, 10, 32, None, 16, None, 1, None, 0, None, None, 1,
                                        None, None, None, None, 0, 1, ctypes.byref(best), None,
                                        None, 0, None) == ann.ANN_EINVAL


def test_grouped_build_rejects_bad_arguments_without_gpu_work():
    from paper_2506_15986_amd import ann
    base = np.zeros((64, 8), np.float32)
    lab = np.zeros((64, 2), np.int32)
    cand = np.zeros((64, 8), np.int32)
    cd2 = np.zeros((64, 8), np.float64)
    ws = np.zeros(256, np.uint8)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731

    def gc(g0=0, g1=1, n_member=2, n_groups=1, k=8, b=base):
        return ann._lib.ann_group_candidates(P(b), 64, 8, k, P(lab), n_member, n_groups, g0, g1,
                                             P(cand), P(cd2), P(ws), ws.nbytes, None)

    assert gc(g0=1, g1=0) == ann.ANN_EINVAL
    assert gc(g1=2) == ann.ANN_EINVAL                 # past n_groups
    assert gc(n_member=0) == ann.ANN_EINVAL
    assert gc(n_groups=0) == ann.ANN_EINVAL
    assert gc(k=0) == ann.ANN_EINVAL
    raw = np.zeros(64 * 8 * 4 + 16, np.uint8)
    assert gc(b=raw[4:4 + 64 * 8 * 4].view(np.float32)) == ann.ANN_EINVAL     # misaligned
    g = np.zeros((64, 4), np.int32)
    m, br = ctypes.c_int32(), (ctypes.c_int32 * 2)()
    # R - 2 <= knn_k, alpha >= 1, R <= 64 (ENOTSUP), workspace size
    assert ann._lib.ann_graph_from_candidates(P(base), 64, 8, P(cand), P(cd2), 1, 4, 1.2, P(g),
                                              ctypes.byref(m), ctypes.byref(br), P(ws), ws.nbytes,
                                              None) == ann.ANN_EINVAL
    assert ann._lib.ann_graph_from_candidates(P(base), 64, 8, P(cand), P(cd2), 8, 4, 0.5, P(g),
                                              ctypes.byref(m), ctypes.byref(br), P(ws), ws.nbytes,
                                              None) == ann.ANN_EINVAL
    assert ann._lib.ann_graph_from_candidates(P(base), 64, 8, P(cand), P(cd2), 8, 65, 1.2, P(g),
                                              ctypes.byref(m), ctypes.byref(br), P(ws), ws.nbytes,
                                              None) == ann.ANN_ENOTSUP
    assert ann._lib.ann_graph_from_candidates(P(base), 64, 8, P(cand), P(cd2), 8, 4, 1.2, P(g),
                                              ctypes.byref(m), ctypes.byref(br), P(ws), ws.nbytes,
                                              None) == ann.ANN_EINVAL      # workspace too small
    assert ann.ann_graph_from_candidates_workspace_size(64, 8, 4) > ws.nbytes
    assert ann.ann_group_candidates_workspace_size(8, 8, 64, 32) > 0
    assert ann.ann_group_candidates_workspace_size(8, 0, 64, 32) == 0


def test_hbkm_rejects_bad_shapes_without_gpu_work():
    from paper_2506_15986_amd import ann
    base = np.zeros((100, 8), np.float32)
    out = np.zeros(4096, np.int32)
    ws = np.zeros(256, np.uint8)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731

    def call(k=4, levels=2, lam=1.0, iters=3, n=100):
        return ann._lib.ann_select_hubs_hbkm(P(base), n, 8, k, levels, lam, iters, P(out), None,
                                             P(out), P(ws), ws.nbytes, None)

    assert call(k=1) == ann.ANN_EINVAL
    assert call(k=65) == ann.ANN_EINVAL
    assert call(levels=0) == ann.ANN_EINVAL
    assert call(k=4, levels=4) == ann.ANN_EINVAL          # 256 clusters > 100 points
    assert call(lam=-1.0) == ann.ANN_EINVAL
    assert call(iters=0) == ann.ANN_EINVAL
    assert call() == ann.ANN_EINVAL                       # workspace too small
    assert ann.ann_select_hubs_hbkm_workspace_size(100, 8, 4, 2) > 256
    assert ann.ann_select_hubs_hbkm_workspace_size(100, 8, 4, 4) == 0


def test_merge_candidates_rejects_bad_widths_without_gpu_work():
    from paper_2506_15986_amd import ann
    base = np.zeros((100, 8), np.float32)
    ids = np.zeros(100 * 1024, np.int32)
    d2 = np.zeros(100 * 1024, np.float64)
    ws = np.zeros(256, np.uint8)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731

    def call(aw=8, bw=8, a=ids, b=ids, wsb=256, n=100):
        return ann._lib.ann_merge_candidates(P(base), n, 8, P(a) if a is not None else None, aw,
                                             P(b) if b is not None else None, bw, P(ids), P(d2),
                                             P(ws), wsb, None)

    assert ann.ann_merge_candidates_workspace_size() == 256
    assert call(aw=0, bw=0) == ann.ANN_EINVAL
    assert call(aw=1000, bw=25) == ann.ANN_EINVAL          # union wider than 1024
    assert call(aw=-1) == ann.ANN_EINVAL
    assert call(a=None) == ann.ANN_EINVAL
    assert call(aw=0, b=None) == ann.ANN_EINVAL
    assert call(wsb=128) == ann.ANN_EINVAL
    assert call(n=0) == ann.ANN_EINVAL


def test_queue_builder_rejects_bad_arguments_on_the_host(lib):
    from paper_2506_15986_amd import ann
    fake = ctypes.c_void_p(0x10000)      # never dereferenced: validation fails first
    tot = (ctypes.c_int64 * 2)()
    wsb = ann.ann_make_queues_workspace_size(300, 70)

    def q(**kw):
        a = dict(hops=fake, nq=300, nh=70, tp=3, tn=15, po=fake, no=fake, pq=None, pc=0, nq_=None,
                 nc=0, ws=fake, wsb=wsb)
        a.update(kw)
        return ann._lib.ann_make_queues(a["hops"], a["nq"], a["nh"], a["tp"], a["tn"], a["po"],
                                        a["no"], a["pq"], a["pc"], a["nq_"], a["nc"], tot, a["ws"],
                                        a["wsb"], None)

    assert q(hops=None) == ann.ANN_EINVAL
    assert q(nq=0) == ann.ANN_EINVAL
    assert q(nh=0) == ann.ANN_EINVAL
    assert q(tp=-1) == ann.ANN_EINVAL
    assert q(pc=5) == ann.ANN_EINVAL              # capacity without a buffer
    assert q(wsb=wsb - 1) == ann.ANN_EINVAL


def test_serving_row_pool_first_fit_and_merge():
    # the serving loop's row allocator: ranges never overlap, freed ranges
    # merge with their neighbours, and the pool's use is the rows held
    import random
    from paper_2506_15986_amd.serve import RowPool
    p = RowPool(100)
    assert p.alloc(30) == 0 and p.alloc(30) == 30 and p.alloc(50) == -1 and p.largest() == 40
    p.release(0, 30)
    assert p.free == [(0, 30), (60, 40)]
    p.release(30, 30)
    assert p.free == [(0, 100)]
    held = []
    rnd = random.Random(1)
    for _ in range(3000):
        if held and rnd.random() < 0.5:
            p.release(*held.pop(rnd.randrange(len(held))))
        else:
            n = rnd.randint(1, 30)
            st = p.alloc(n)
            if st >= 0:
                assert all(st + n <= a or a + b <= st for a, b in held)
                held.append((st, n))
        fr = p.free
        assert all(fr[i][0] + fr[i][1] < fr[i + 1][0] for i in range(len(fr) - 1))
        assert p.in_use() == sum(b for _, b in held)


def test_noalloc_search_rejects_bad_arguments_on_the_host(lib):
    from paper_2506_15986_amd import ann
    fake = ctypes.c_void_p(0x10000)      # never dereferenced: validation fails first
    big = ann.ANN_NOALLOC_MAX_QUERIES + 1
    st = ann._lib.ann_search_noalloc(fake, 1000, 32, fake, 16, fake, big, None, 0, fake, fake, 10,
                                     fake, fake, None, None, 0, None, None)
    assert st == ann.ANN_EINVAL and "at most" in ann.last_error()
    st = ann._lib.ann_search_noalloc(fake, 1000, 32, fake, 16, fake, -1, None, 0, fake, fake, 10,
                                     fake, fake, None, None, 0, None, None)
    assert st == ann.ANN_EINVAL


def test_seeded_hub_start_matches_oracle_on_the_host(lib):
    import oracle
    from paper_2506_15986_amd import ann
    for n, m, seed in ((10, 10, 3), (1_000_000, 1024, 0), (20_000, 64, 2**63 + 5), (7, 1, 1),
                       (10_000_000, 1024, 12345)):
        got = ann.ann_hub_init_ids(n, m, seed).numpy()
        assert (got == oracle.hub_init_ids(n, m, seed)).all(), (n, m, seed)
    out = (ctypes.c_int32 * 4)()
    assert ann._lib.ann_hub_init_ids(3, 4, 0, out) == ann.ANN_EINVAL        # n_hubs > n
    assert ann._lib.ann_hub_init_ids(3, 0, 0, out) == ann.ANN_EINVAL
    assert ann._lib.ann_hub_init_ids(2**31, 4, 0, out) == ann.ANN_EINVAL
    assert ann._lib.ann_hub_init_ids(10, 4, 0, None) == ann.ANN_EINVAL


def test_entry_model_handle_checks_fields_on_the_host(lib):
    from paper_2506_15986_amd import ann
    fake = 0x10000                       # never dereferenced
    tw = ann.ann_tower(din=128, hidden=256, dout=64, in_scale=1.0, W1=fake, b1=fake, W2=fake,
                       b2=fake, W1b=fake, W2b=fake)

    def make(**kw):
        a = dict(query_tower=tw, hub_emb=fake, hub_graph=fake, n_hubs=1024, s=16, hub_ids=fake,
                 hub_entry=3, medoid=7, L_h=48, theta=float("-inf"),
                 hub_plan=ann.ann_search_plan())
        a.update(kw)
        return ann.ann_entry_model(**a)

    h = ctypes.POINTER(ann.ann_entry_model)()
    desc = make()
    assert ann._lib.ann_entry_model_create(ctypes.byref(desc), ctypes.byref(h)) == ann.ANN_OK
    assert h.contents.n_hubs == 1024 and h.contents.L_h == 48 and h.contents.hub_entry == 3
    assert h.contents.hub_emb == fake and h.contents.query_tower.dout == 64
    desc.L_h = 5                          # a copy: the handle keeps its own fields
    assert h.contents.L_h == 48
    ann._lib.ann_entry_model_destroy(h)
    ann._lib.ann_entry_model_destroy(None)
    for kw, code in ((dict(hub_emb=None), ann.ANN_EINVAL), (dict(hub_entry=1024), ann.ANN_EINVAL),
                     (dict(L_h=0), ann.ANN_EINVAL), (dict(L_h=513), ann.ANN_EINVAL),
                     (dict(s=65), ann.ANN_ENOTSUP), (dict(medoid=-1), ann.ANN_EINVAL),
                     (dict(hub_emb=fake + 4), ann.ANN_EINVAL),
                     (dict(hub_plan=ann.make_plan(pool_cap=64, group=12)), ann.ANN_EINVAL)):
        h = ctypes.POINTER(ann.ann_entry_model)()
        d = make(**kw)
        assert ann._lib.ann_entry_model_create(ctypes.byref(d), ctypes.byref(h)) == code, kw
        assert not h
    assert ann._lib.ann_entry_model_create(None, ctypes.byref(h)) == ann.ANN_EINVAL
