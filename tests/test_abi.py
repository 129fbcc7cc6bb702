"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments on the host before touching the device (CPU only)."""
import ctypes
import os
import re

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

    def call(**kw):
        a = dict(base=fake, n=1000, dim=32, graph=fake, R=16, queries=fake, nq=4, entry=None,
                 medoid=0, k=fake, L=fake, k_max=10, ids=fake, dist=fake, stats=None, trace=None,
                 trace_cap=0, plan=None, ws=fake, wsb=256, stream=None)
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
    assert call(k_max=0) == ann.ANN_EINVAL
    bad = ann.ann_search_plan(pool_cap=1024, visited_log2=12, group=8, waves_per_block=1,
                              blocks=0, fp64=0)
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    bad.pool_cap, bad.group = 64, 12
    assert call(plan=ctypes.byref(bad)) == ann.ANN_EINVAL
    # nq == 0 is valid and enqueues nothing
    assert call(nq=0) == ann.ANN_OK


def test_default_plan_and_workspace():
    from paper_2506_15986_amd import ann
    p = ann.default_plan(1_000_000, 128, 32, 200)
    assert p.pool_cap == 256 and p.group == 8 and p.fp64 == 0
    p = ann.default_plan(1_000_000, 960, 64, 400)
    assert p.pool_cap == 512 and p.group == 16
    with pytest.raises(ann.AnnError):
        ann.default_plan(10, 32, 16, 600)
    assert ann.workspace_size("search", 1000, 32, 10) >= 4


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
