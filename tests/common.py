"""Shared fixtures for the GPU parity tests: seeded workloads and the oracle's
index for them (built once per session, on the CPU)."""
import functools
import sys

import numpy as np

import oracle
from paper_2506_15986_amd import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def tiny_index(n=10_000, nq=100):
    """The tiny workload (10k x 32 Gaussian mixture on the 2^-19 grid), its
    kNN(64) -> alpha 1.2 -> R=16 graph, medoid and exact top-10."""
    w = synth.scaled(synth.WORKLOADS["tiny"], n=n, n_queries=nq)
    base = synth.base(w)
    q = synth.queries(w)
    g, med, nf, nr, cand, cd2 = oracle.build_graph(base, knn_k=64, R=16, alpha=1.2)
    truth, td2 = oracle.knn(base, q, 10)
    return dict(w=w, base=base, q=q, graph=g, medoid=med, cand=cand, cand_d2=cd2,
                truth=truth, truth_d2=td2, nf=nf, nr=nr)


@functools.lru_cache(maxsize=None)
def int_index(n=20_000, nq=200, R=32, knn_k=64):
    """Integer-valued data (the 1M x 128 recipe at reduced N: values 0..255),
    where FP32 squared distances are exact."""
    w = synth.scaled(synth.WORKLOADS["sift1m"], n=n, n_queries=nq)
    base = synth.base(w)
    q = synth.queries(w)
    g, med, nf, nr, cand, cd2 = oracle.build_graph(base, knn_k=knn_k, R=R, alpha=1.2)
    truth, td2 = oracle.knn(base, q, 10)
    return dict(w=w, base=base, q=q, graph=g, medoid=med, cand=cand, cand_d2=cd2,
                truth=truth, truth_d2=td2, nf=nf, nr=nr)


def first_divergence(tr_a, tr_b):
    """Index of the first differing expansion of two traces (or -1)."""
    m = min(len(tr_a), len(tr_b))
    for t in range(m):
        if tr_a[t] != tr_b[t]:
            return t
    return -1 if len(tr_a) == len(tr_b) else m


def near_tie_certificate(base, graph, q, entry, L, tr_gpu, tr_cpu, tol=1e-5):
    """Divergence certificate for an FP32 search against the FP64 oracle.

    Up to the first differing expansion both sides expanded the same nodes, so
    they saw the same visited set S and each pool is the L best keys of S under
    its own distances.  The two choices can then differ only through a near
    tie: between the two chosen nodes, or between a chosen node and the L-th
    best exact key of S (pool admission).  Returns True when the first
    difference is such a tie within `tol` (relative)."""
    tr_gpu = [int(x) for x in tr_gpu if x >= 0]
    tr_cpu = [int(x) for x in tr_cpu if x >= 0]
    t = first_divergence(tr_gpu, tr_cpu)
    if t < 0:
        return True
    seen = {int(entry)}
    for p in tr_cpu[:t]:
        seen.update(int(v) for v in graph[p] if v >= 0)
    keys = sorted(oracle.sqdist(q, base[v]) for v in seen)
    kL = keys[L - 1] if len(keys) >= L else float("inf")

    def close(x, y):
        return abs(x - y) <= tol * max(abs(x), abs(y), 1e-30)

    picks = [oracle.sqdist(q, base[v]) for v in
             (tr_gpu[t] if t < len(tr_gpu) else None, tr_cpu[t] if t < len(tr_cpu) else None)
             if v is not None]
    if len(picks) == 2 and close(picks[0], picks[1]):
        return True
    return any(close(d, kL) for d in picks)


def tower_certificate(params, x, e_gpu, in_scale=1.0, tol=1e-4):
    """Checks GPU tower embeddings against the oracle's (FP64 on the same BF16
    operands).  Derivation of the tolerance: the BF16 x BF16 products are
    exact in FP32, so the GPU's first-layer pre-activation z1 differs from the
    FP64 one only by FP32 summation error, at most eps_j = (K + 2) 2^-24
    (sum_k |x_k w_jk| + |b_j|) over K inputs; the second layer and the
    normalisation add errors of the same relative size (~1e-6), far below
    tol = 1e-4 on the unit row (L2 norm of the difference).  The one step
    that can amplify them is the re-rounding of the hidden activation to
    BF16: where relu(z1_j) lies within eps_j of a rounding boundary the GPU
    may round it to the neighbouring BF16 value (one ulp, 2^-8 relative),
    which moves the output row by up to (2 / |z2|) |delta a_j| |W2[:, j]|.
    A row beyond tol is certified when its error is within tol plus that
    bound summed over its ambiguous hidden elements.

    Returns (rows beyond tol, rows certified by ambiguous roundings, indices
    of uncertified rows)."""
    from oracle import towers as T
    e_ref, c = T.tower_forward(params, x, bf16=True, in_scale=in_scale)
    e_gpu = np.asarray(e_gpu, np.float64)
    err = np.linalg.norm(e_gpu - e_ref, axis=1)
    bad = np.flatnonzero(err > tol)
    if bad.size == 0:
        return 0, 0, []
    b1 = np.asarray(params[1], np.float64)
    b2 = np.asarray(params[3], np.float64)
    xr, W1r, W2r = c["xr"], c["W1r"], c["W2r"]
    K = xr.shape[1]
    col = np.linalg.norm(W2r, axis=0)                 # |W2[:, j]|
    unc, cert = [], 0
    for i in bad:
        eps = (K + 2) * 2.0 ** -24 * (np.abs(xr[i]) @ np.abs(W1r).T + np.abs(b1))
        z = c["z1"][i]
        lo = T.bf16_round(np.maximum(z - eps, 0.0))
        hi = T.bf16_round(np.maximum(z + eps, 0.0))
        amb = np.abs(hi - lo)
        z2 = c["a1r"][i] @ W2r.T + b2
        bound = tol + 2.0 / np.linalg.norm(z2) * float((amb * col).sum())
        if err[i] <= bound and amb.any():
            cert += 1
        else:
            unc.append(int(i))
    return int(bad.size), cert, unc


def hub_search_traced(ann, gm, qe_sub, L_h):
    """The entry stage's hub search re-run with traces on some query
    embeddings (the register-pool search when L_h <= 64, else the base search
    kernel with the model's hub plan, as ann_entry_select picks them).
    Returns (best hub indices, traces) on the host."""
    if L_h <= 64:
        b, _, _, tr = ann.ann_hub_search(gm.hub_emb, gm.hub_graph, qe_sub, gm.hub_entry, L_h,
                                         trace_cap=1024)
        return b.cpu().numpy(), tr.cpu().numpy()
    ids, _, _, tr = ann.ann_search(gm.hub_emb, gm.hub_graph, qe_sub, None, gm.hub_entry, 1, L_h,
                                   plan=gm.model.c.hub_plan, trace_cap=1024)
    return ids.cpu().numpy()[:, 0], tr.cpu().numpy()
