"""Benchmark: QPS at recall@10 = 0.95 of the GATE query path on one MI355X,
GATE entry vs medoid entry.

Workload (default, "sift1m"): 1,000,000 x 128 base vectors holding integers
0..255 (256-component Gaussian mixture, sigma 20), 10,000 test queries and
100,000 training queries from the same mixture.  Index: exact 128-NN ->
alpha 1.2 pruning -> R = 32 with connectivity repair; 1,024 Lloyd hubs; two
towers 128->128->64 and (128+32)->128->64 trained with the contrastive loss;
hub navigation graph s = 16.  All of it is built on the GPU before timing.

One step = the whole query path over the 10,000-query batch, inputs resident
in HBM: entry selection (query tower + hub-graph search) then the batched
beam search, each stage one HIP-graph replay, the search with the plan the
autotuner picked on this batch.  The K timed steps run pipelined on two
streams: the entry stage of batch i+1 runs beside the search of batch i (two
sets of buffers, events order each batch's search after its entry stage); the
same steps run back to back are reported too (qps_sequential), and the
search kernel's roofline comes from the back-to-back launches.  The beam width L is the smallest on the
sweep whose mean recall@10 reaches 0.95.  The medoid entry is measured the
same way (search stage only); when it never reaches 0.95 its best recall and
the QPS there are reported.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --save-state DIR            # also keep the built index/model
    python bench.py --load-state DIR --legs gate --no-cpu   # serve a saved build

The --load-state form replays the same timed GATE step without rebuilding or
sweeping; it is the command the kernel profiles are taken on, so that the
profiler sees only the timed launches.  Prints one compact JSON line on
stdout, last (the headline, the medoid comparison, the roofline and the CPU
oracle's rate and its query-by-query parity with the GPU's batch); the full
record (sweeps, autotune rows, ablations, serving) goes to --details;
progress goes to stderr (one line per swept width with --verbose).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QPS at recall@10=0.95, GATE entry vs medoid entry, 1M×128 on one MI355X"
HBM_PEAK_GBS = 8000.0
TARGET = 0.95
L_SWEEP = ([10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56] + list(range(64, 257, 8)) +
           [288, 320, 384, 448, 512])
SEARCH_SOURCES = ("search.hip", "search_core.h", "beam.h")
WORKLOAD_TEXT = {
    "sift1m": "integers 0..255 (256-component GMM, sigma 20)",
    "shift1m": "unit-normalised (512-component GMM); test and training queries from means shifted "
               "by 0.3 sigma with Dirichlet(0.3) cluster weights",
    "gist1m": "256-component GMM with LogNormal(0, 0.5) per-dimension scales; half the queries "
              "mean-shifted",
    "tiny": "16-component GMM, sigma 1",
    "sift10m": "integers 0..255 (256-component GMM, sigma 20); 30% of the queries mean-shifted",
}
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def search_source_hash() -> str:
    """Digest of the search kernel's sources with comments and blank space
    removed: counter figures taken on another version of the kernel's code
    are not reported (a comment edit keeps them)."""
    h = hashlib.sha256()
    for f in SEARCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2506_15986_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, L: int, nq: int, plan: dict):
    """HBM bytes per search launch (reads, writes) from the committed counter
    summary, when it was taken on this kernel version, workload, L, batch and
    plan.  The plan must agree in gather group, filter form and size; the
    wavefronts per workgroup only change how waves are packed, not what a
    query reads, so they are not compared."""
    path = os.path.join(ROOT, "profiles", "search_kernel_%s.md" % workload)
    if not os.path.exists(path):
        return None
    want = dict(kernel_hash=search_source_hash(), L=str(L), nq=str(nq))
    for line in open(path):
        m = re.match(r"^traffic:\s*(.*)$", line.strip())
        if not m:
            continue
        kv = dict(p.split("=", 1) for p in m.group(1).split() if "=" in p)
        pl = kv.get("plan", "").split("/")
        if (all(kv.get(a) == b for a, b in want.items()) and len(pl) == 4 and
                pl[0] == str(plan["group"]) and pl[1] == str(plan["visited_log2"]) and
                pl[3] == str(plan["filter"]) and plan.get("waves_per_query", 1) in (0, 1)):
            return float(kv["read_bytes"]), float(kv["write_bytes"])
    return None


def host_cpu() -> dict:
    """Host processor model and online core count (from /proc/cpuinfo)."""
    model, n = "", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = model or line.split(":", 1)[1].strip()
                n += 1
    except OSError:
        pass
    return dict(model=model, logical_cpus=n or os.cpu_count())


def recall_at(ids: np.ndarray, truth: np.ndarray, k: int = 10) -> np.ndarray:
    """Eq. 1 recall per query, ground truth ordered by (distance, id)."""
    hit = (ids[:, :k, None] == truth[:, None, :k]).any(-1)
    return hit.sum(1) / float(k)


def recall_tie_aware(dist: np.ndarray, truth_dist: np.ndarray, k: int = 10) -> np.ndarray:
    """A returned point counts when its distance is within the k-th true one
    (up to the 1e-5 relative tolerance between FP32 search distances and the
    ground truth's)."""
    lim = truth_dist[:, k - 1:k].astype(np.float64)
    return (dist[:, :k].astype(np.float64) <= lim + 1e-5 * np.maximum(lim, 1e-6)).sum(1) / float(k)


def finite(x):
    """The value with every non-finite float replaced by None, so that the
    summary line is strict JSON (a medoid-fallback threshold of -inf means
    "never falls back")."""
    if isinstance(x, float):
        return x if np.isfinite(x) else None
    if isinstance(x, dict):
        return {k: finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite(v) for v in x]
    return x


def serving_summary(sv):
    """The serving leg's headline figures for the summary line."""
    if not sv:
        return None
    half = next((x for x in sv["loads"] if abs(x["offered_qps"] / sv["capacity_qps"] - 0.5) < 0.05),
                None)
    return dict(capacity_qps=sv["capacity_qps"], theta=sv["theta"], fallbacks=sv["fallbacks"],
                half_load=dict(qps=half["qps"], p50_ms=half["p50_ms"], p99_ms=half["p99_ms"],
                               served_recall=half["served_recall"]) if half else None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sift1m")
    ap.add_argument("--n", type=int, default=0, help="override base size")
    ap.add_argument("--n-train", type=int, default=0, help="override training-query count")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--select-epoch", action="store_true",
                    help="keep the towers of the epoch with the best held-out label agreement "
                         "(--epochs is then a budget)")
    ap.add_argument("--R", type=int, default=32, help="graph out-degree")
    ap.add_argument("--knn-k", type=int, default=128, help="kNN candidates before pruning")
    ap.add_argument("--alpha", type=float, default=1.2, help="pruning parameter of the graph")
    ap.add_argument("--partitions", type=int, default=0,
                    help="candidate lists from this many overlapping k-means groups instead of "
                         "the all-pairs kNN (0: all pairs)")
    ap.add_argument("--overlap", type=int, default=2, help="groups listed per point")
    ap.add_argument("--hubs", type=int, default=1024)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--dout", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tau", type=float, default=0.07)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--legs", default="medoid,gate,ablation,serve",
                    help="also: hbkm (GATE on hierarchical balanced k-means hubs, one model per "
                         "--hbkm-lambdas value), queues (GATE trained on Definition 4 queues with "
                         "the hub-anchored Eq. 4 loss), fusion (GATE with the Eq. 3 fusion embedding), "
                         "nsg (medoid and GATE on an NSG-style graph)")
    ap.add_argument("--hbkm-lambdas", default="0,1,10")
    ap.add_argument("--nsg-L", default="128",
                    help="nsg leg: beam widths of the per-point build searches, one graph each")
    ap.add_argument("--nsg-path", type=int, default=0,
                    help="nsg leg: also take the first this many expanded nodes of each build "
                         "search as candidates")
    ap.add_argument("--queue-variants", default="3:16:48",
                    help="queues leg: t_pos:P:N triples, comma separated (t_neg stays 15)")
    ap.add_argument("--no-tune", action="store_true", help="time the default plan")
    ap.add_argument("--pipe", type=int, default=2, help="searches in flight in the pipelined steps")
    ap.add_argument("--pipe-buffers", type=int, default=0,
                    help="buffer sets of the pipelined steps (0: one more than the searches in "
                         "flight, so that a batch's entry stage runs ahead of its search)")
    ap.add_argument("--pipe-replay", action="store_true",
                    help="with --load-state, also time the pipelined steps")
    ap.add_argument("--shuffle-queries", type=int, default=0,
                    help="permute the test queries with this seed (0: generator order)")
    ap.add_argument("--save-state", default="")
    ap.add_argument("--load-state", default="")
    ap.add_argument("--details", default=os.path.join("gpurun_out", "bench_details.json"),
                    help="file for the full record (sweeps, autotune rows, ablations); the stdout "
                         "line carries the summary only ('' = do not write)")
    ap.add_argument("--verbose", action="store_true", help="one progress line per swept width")
    ap.add_argument("--targets", default="0.95",
                    help="recall@10 targets to report (the headline is 0.95)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; multi-GPU runs are not part of this build "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    PIPE = max(2, args.pipe)
    NBUF = max(PIPE, args.pipe_buffers) if args.pipe_buffers else PIPE + 1
    targets = sorted(set([TARGET] + [float(x) for x in args.targets.split(",") if x]))

    import torch

    from paper_2506_15986_amd import ann, gate, synth

    dev = torch.device("cuda:0")
    w = synth.WORKLOADS[args.workload]
    if args.n or args.n_train:
        w = synth.scaled(w, n=args.n or None, n_train=args.n_train or None)
    knn_k, R, k = args.knn_k, args.R, 10
    parts = args.partitions

    t0 = time.time()
    base = synth.base(w)
    queries = synth.queries(w)
    if args.shuffle_queries:
        queries = queries[np.random.default_rng(args.shuffle_queries).permutation(queries.shape[0])]
    log("data: %d x %d base, %d queries (%.1fs)" % (w.n, w.d, queries.shape[0], time.time() - t0))
    base_d = torch.from_numpy(base).to(dev)
    q_d = torch.from_numpy(queries).to(dev)
    nq = q_d.shape[0]

    state = None
    if args.load_state:
        index, g, state = gate.load_state(args.load_state, base_d)
        log("state loaded from %s: medoid %d, L gate %s, L medoid %s" %
            (args.load_state, index.medoid, state.get("L_gate"), state.get("L_medoid")))
    else:
        index = gate.build_index(base_d, knn_k, R, args.alpha, partitions=parts, overlap=args.overlap,
                                 w=w, log=log)
        g = None
    log("graph: kNN %d%s -> alpha %g -> R %d, medoid %d, bridges %s (%.1fs)" %
        (knn_k, " in %d groups x %d" % (parts, args.overlap) if parts else "", args.alpha, R,
         index.medoid,
         index.bridges, index.build_s))
    gt_ids, gt_dist = ann.ann_gt_knn(base_d, q_d, k)
    gt, gtd = gt_ids.cpu().numpy(), gt_dist.cpu().numpy()

    kk = torch.full((nq,), k, dtype=torch.int32, device=dev)
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
           torch.empty((nq, k), dtype=torch.float32, device=dev),
           torch.empty((nq, 4), dtype=torch.int32, device=dev))
    ws = ann.workspace("search", w.n, w.d, nq, device=dev)

    def sweep(entry, label):
        """recall@10 over the L grid until the largest target is reached; the
        first grid width that reaches the headline target is refined in
        steps of 8 from the grid width below it."""
        rows, L95 = [], None

        def measure(L):
            index.search(q_d, L, kk, entry, out=out, ws=ws)
            torch.cuda.synchronize()
            rec = float(recall_at(out[0].cpu().numpy(), gt).mean())
            st = out[2].cpu().numpy()
            rows.append(dict(L=L, recall=round(rec, 5), ndc=round(float(st[:, 0].mean()), 1),
                             hops=round(float(st[:, 2].mean()), 1)))
            if args.verbose:
                log("  %s L=%4d recall@10=%.4f ndc=%.0f hops=%.0f" % (label, L, rec, st[:, 0].mean(),
                                                                      st[:, 2].mean()))
            return rec

        prev = None
        for L in L_SWEEP:
            rec = measure(L)
            if rec >= TARGET and L95 is None:
                for Lr in range(prev + 8, L, 8) if prev is not None else ():
                    if measure(Lr) >= TARGET:
                        L95 = Lr
                        break
                if L95 is None:
                    L95 = L
            if rec >= max(targets):
                break
            prev = L
        rows.sort(key=lambda r: r["L"])
        best = max(rows, key=lambda r: r["recall"])
        log("sweep %s: %d widths, L for recall %.2f: %s, best recall %.4f at L = %d" %
            (label, len(rows), TARGET, L95, best["recall"], best["L"]))
        return rows, L95

    def extra_targets(rows, model, entry, label):
        """QPS at the other recall targets (their smallest L on the sweep)."""
        out = []
        for t in targets:
            if t == TARGET:
                continue
            Lt = next((r["L"] for r in rows if r["recall"] >= t), None)
            rec = dict(target=t, L=Lt)
            if Lt is not None:
                r = timed(Lt, model, entry, "%s@%g" % (label, t))
                rec.update(recall=r["recall"], qps=r["qps"], search_ms=r["search_ms"],
                           entry_ms=r["entry_ms"], ndc=r["ndc"])
            out.append(rec)
        return out

    def tune(L, entry, label):
        if state is not None and state.get("plan_%s" % label):
            return ann.make_plan(**state["plan_%s" % label]), []
        if args.no_tune:
            return ann.default_plan(w.n, w.d, R, L), []
        t = time.time()
        best, times = ann.ann_autotune_search(base_d, index.graph, q_d, entry, index.medoid, kk,
                                              torch.full((nq,), L, dtype=torch.int32, device=dev),
                                              k, L, reps=3)
        rows = [dict(p.as_dict(), ms=round(ms, 4)) for p, ms in times]
        log("autotune %s L=%d: %d plans in %.1fs, best %s (%.3f ms; default %.3f ms)" %
            (label, L, len(times), time.time() - t, best,
             min(ms for _, ms in times if ms >= 0), times[0][1]))
        return best, rows

    def pipe_candidates(plan, rows, label):
        """Search plans tried for the pipelined steps.  With two batches in
        flight the next search's wavefronts and the entry stage need compute
        units while the current search still runs, so a persistent grid that
        fills the GPU is not always best there: the tuned plan and the best
        plan of the other gather group (from the single-launch autotuner's
        rows) are each tried with their own and with four wavefronts per
        workgroup, with the full grid and with grids of 16 down to 12
        wavefronts per compute unit."""
        if state is not None and state.get("pipe_plan_%s" % label):
            return [ann.make_plan(**state["pipe_plan_%s" % label])]
        if state is not None or args.no_tune:
            return [plan]
        bases = [plan]
        other = sorted((r for r in rows if r["group"] != plan.group and r["ms"] >= 0
                        and r.get("waves_per_query", 1) == 1), key=lambda r: r["ms"])
        if other:
            bases.append(ann.make_plan(**{f: v for f, v in other[0].items() if f != "ms"}))
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        out = []
        for bp in bases:
            own = max(1, int(bp.waves_per_block))
            # several wavefronts per query fix the workgroup at that many
            for wpb in sorted({own, 4}) if int(bp.waves_per_query) <= 1 else [own]:
                for wpc in (0, 16, 15, 14, 13, 12):
                    out.append(ann.make_plan(**dict(bp.as_dict(), waves_per_block=wpb,
                                                    blocks=(wpc * cus) // wpb)))
        return out

    def pipelined(b, L, plan, model, rows, label):
        """The same K steps with PIPE searches in flight: the entry stage runs
        on its own stream, and the searches of consecutive batches on PIPE
        streams in turn, so the next batch's search fills the compute units
        that the current one's last queries leave idle.  NBUF buffer sets
        (PIPE + 1 by default) are used in turn; events order each buffer's
        entry stage after the last search on those buffers and each search
        after its entry stage.  With PIPE buffer sets the entry stage of a
        batch waits for the search two batches back and then for compute
        units beside the other stream's running search, which could hold
        every other step back; one more set lets it run a step ahead.  With the tail filled that way, the
        searches take their queries as given (plan.query_order), which
        measured faster here than widest-expected-first.  The search plan is
        the fastest of pipe_candidates over a short pipelined run (35 steps
        each); every candidate's results are compared with the timed batch's."""
        # streams with hardware queues of their own: on ordinary streams the
        # two searches may share a queue and then run one after the other
        s_e = ann.dedicated_stream(0, dev)
        s_s = [ann.dedicated_stream(1 + x, dev) for x in range(PIPE)]

        def run(cand, steps, warmup):
            pplan = ann.make_plan(**dict(cand.as_dict(), query_order=ann.ANN_ORDER_AS_GIVEN))
            extra = [ann.QueryBatch(base_d, index.graph, index.medoid, q_d, kk,
                                    torch.full((nq,), L, dtype=torch.int32, device=dev), k,
                                    plan=pplan, model=model,
                                    entry_ids=None if model is not None else b.entry_ids)
                     for _ in range(NBUF)]
            pairs = [(bx.graph_exec(ann.ANN_STAGE_ENTRY) if model is not None else None,
                      bx.graph_exec(ann.ANN_STAGE_SEARCH)) for bx in extra]
            ready = [torch.cuda.Event() for _ in range(NBUF)]
            done = [torch.cuda.Event() for _ in range(NBUF)]
            for x in range(NBUF):
                done[x].record(s_s[x % PIPE])

            def pstep(i):
                # buffer set i % NBUF, search stream i % PIPE: a stream runs its
                # searches in order, so at most PIPE are in flight, and with one
                # buffer set more than that a batch's entry stage waits only for
                # the search before the previous one on its buffers
                x, ss = i % NBUF, s_s[i % PIPE]
                ge, gs = pairs[x]
                if ge is not None:
                    s_e.wait_event(done[x])
                    ge.launch(stream=s_e)
                    ready[x].record(s_e)
                    ss.wait_event(ready[x])
                gs.launch(stream=ss)
                done[x].record(ss)

            for i in range(warmup):
                pstep(i)
            torch.cuda.synchronize()
            t0 = time.time()
            for i in range(steps):
                pstep(i)
            torch.cuda.synchronize()
            wall = time.time() - t0
            same = all(bool((bx.ids.cpu().numpy() == b.ids.cpu().numpy()).all()) for bx in extra)
            for pr in pairs:
                for gx in pr:
                    if gx is not None:
                        gx.close()
            del extra
            return wall * 1000.0 / steps, same

        cands = pipe_candidates(plan, rows, label)
        trials = []
        best = cands[0]
        if len(cands) > 1:
            for cand in cands:
                ms, same = run(cand, 35, 5)
                trials.append(dict(group=int(cand.group), waves_per_block=int(cand.waves_per_block),
                                   visited_log2=int(cand.visited_log2), blocks=int(cand.blocks),
                                   ms_per_step=round(ms, 4), results_equal=same))
            ok = [(t["ms_per_step"], i) for i, t in enumerate(trials) if t["results_equal"]]
            best = cands[min(ok)[1]] if ok else plan
            log("pipelined plan: %d candidates, best group %d, %d waves/workgroup, %d workgroups "
                "(%.3f ms/step; full grid of the tuned plan %.3f)" %
                (len(cands), best.group, best.waves_per_block, best.blocks,
                 min(t["ms_per_step"] for t in trials), trials[0]["ms_per_step"]))
        ms, same = run(best, args.steps, args.warmup)
        res = dict(qps=round(nq * 1000.0 / ms, 1), ms_per_step=round(ms, 4), results_equal=same,
                   plan=best.as_dict(), candidates=trials)
        res["batches_in_flight"] = PIPE
        res["buffer_sets"] = NBUF
        log("pipelined steps (%d batches in flight): %.3f ms/step -> %.0f QPS (results equal: %s)" %
            (PIPE, res["ms_per_step"], res["qps"], same))
        return res

    def timed(L, model, entry, label):
        """K timed steps of HIP-graph replays: [entry stage] + search stage."""
        plan, tune_rows = tune(L, entry, label)
        b = ann.QueryBatch(base_d, index.graph, index.medoid, q_d, kk,
                           torch.full((nq,), L, dtype=torch.int32, device=dev), k, plan=plan,
                           model=model, entry_ids=None if model is not None else entry)
        g_entry = b.graph_exec(ann.ANN_STAGE_ENTRY) if model is not None else None
        g_search = b.graph_exec(ann.ANN_STAGE_SEARCH)

        def step(ev=None):
            if ev:
                ev[0].record()
            if g_entry is not None:
                g_entry.launch()
            if ev:
                ev[1].record()
            g_search.launch()
            if ev:
                ev[2].record()

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        t0 = time.time()
        for ev in evs:
            step(ev)
        torch.cuda.synchronize()
        wall = time.time() - t0
        search_ms = [e[1].elapsed_time(e[2]) for e in evs]
        entry_ms = [e[0].elapsed_time(e[1]) for e in evs]
        pipe = (pipelined(b, L, plan, model, tune_rows, label)
                if state is None or args.pipe_replay else None)
        ids, dist = b.ids.cpu().numpy(), b.dist.cpu().numpy()
        rec = float(recall_at(ids, gt).mean())
        rec_t = float(recall_tie_aware(dist, gtd).mean())
        st = b.stats.cpu().numpy()
        # exact distance and hop counts of the same searches: a filter large
        # enough not to forget (only the executed count depends on the filter)
        exact = ann.make_plan(**dict(plan.as_dict(), visited_log2=13, filter=ann.ANN_FILTER_ID32,
                                     waves_per_block=1, waves_per_query=1))
        e = b.entry_ids if model is not None else entry
        xs = ann.ann_search(base_d, index.graph, q_d, e, index.medoid, kk, b.L, k_max=k,
                            plan=exact)[2].cpu().numpy()
        d = w.d
        ex = dict(lossy=int(((xs[:, 3] & 1) != 0).sum()), ndc=float(xs[:, 0].mean()),
                  hops=float(xs[:, 2].mean()),
                  bytes=float((4 * d * xs[:, 0].astype(np.float64) +
                               4 * R * xs[:, 2].astype(np.float64) + 4 * d + 8 * k).sum()))
        exacts[label] = ex
        arrays[label] = dict(ids=ids, dist=dist, ndc=xs[:, 0].copy(), hops=xs[:, 2].copy(),
                             entry=(e.cpu().numpy() if e is not None
                                    else np.full(nq, index.medoid, np.int32)))
        lossy, bytes_launch = ex["lossy"], ex["bytes"]
        sm = float(np.mean(search_ms))
        res = dict(L=L, recall=round(rec, 5), recall_tie_aware=round(rec_t, 5),
                   qps=round(nq * args.steps / wall, 1),
                   ms_per_step=round(wall * 1000.0 / args.steps, 4),
                   search_ms=round(sm, 4), search_ms_median=round(float(np.median(search_ms)), 4),
                   entry_ms=round(float(np.mean(entry_ms)), 4),
                   ndc=round(ex["ndc"], 1), hops=round(ex["hops"], 1),
                   ndc_exec=round(float(st[:, 1].mean()), 1), filter_overflow_queries=lossy,
                   plan=plan.as_dict(), bytes_per_launch=bytes_launch,
                   achieved_gbs=round(bytes_launch / (sm / 1000.0) / 1e9, 1), autotune=tune_rows)
        if pipe is not None:
            # the step throughput: batches pipelined over two streams (entry of
            # batch i+1 beside the search of batch i); the sequential figures
            # stay in qps_sequential / ms_per_step_sequential
            res["qps_sequential"], res["ms_per_step_sequential"] = res["qps"], res["ms_per_step"]
            res["qps"], res["ms_per_step"] = pipe["qps"], pipe["ms_per_step"]
            res["pipelined"] = pipe
        log("timed %s: L=%d recall=%.4f (tie-aware %.4f) %.3f ms/step (entry %.3f, search %.3f ms)"
            " -> %.0f QPS, %.0f GB/s, plan %s" %
            (label, L, rec, rec_t, res["ms_per_step"], res["entry_ms"], sm, res["qps"],
             res["achieved_gbs"], plan))
        g_search.close()
        if g_entry is not None:
            g_entry.close()
        return res

    def serving(gm, L):
        """Continuous batching under Poisson arrivals.  Requests of 1..512
        queries from the same mixture with 30 % drawn around shifted means
        (out of distribution), k = 10 or 100 (even odds), each k with the
        smallest L on a sweep of the mix whose recall@k reaches 0.95; GATE
        entries (no fallback).  The capacity is the throughput with every
        request waiting at the start; Poisson arrivals are then offered at
        half and 80 % of it.
        Reports throughput, p50/p99 latency and the served recall@k."""
        import dataclasses

        from paper_2506_15986_amd import serve
        wm = dataclasses.replace(w, shift=0.3, shifted_frac=0.3)
        qm = synth.queries(wm)
        qm_d = torch.from_numpy(qm).to(dev)
        gt100 = ann.ann_gt_knn(base_d, qm_d, 100)[0].cpu().numpy()
        model = gm.model
        # the medoid fallback's threshold, tuned on 10,000 training queries
        # of the same mix at the headline width
        tq_mix = torch.from_numpy(synth.train_queries(wm, 10000)).to(dev)
        theta, theta_rows = gate.tune_theta(index, gm, tq_mix, ann.ann_gt_knn(base_d, tq_mix, 10)[0],
                                            L)
        log("serving: medoid fallback threshold %s (recall@10 at L=%d per threshold, fallbacks: %s)"
            % (theta, L, theta_rows))
        del tq_mix
        em = ann.ann_entry_select(model, qm_d)[0]
        nqm = qm.shape[0]
        Lk = {}
        for kq, grid in ((10, [L] + [x for x in L_SWEEP if x > L]),
                         (100, [x for x in L_SWEEP if x >= 100] + [640, 768, 896, 1024])):
            kt = torch.full((nqm,), kq, dtype=torch.int32, device=dev)
            Lk[kq] = None
            for Lx in grid:
                ids = index.search(qm_d, Lx, kt, em)[0].cpu().numpy()
                rec = float((ids[:, :kq, None] == gt100[:, None, :kq]).any(-1).mean())
                if args.verbose:
                    log("  serving mix k=%d L=%d recall@%d=%.4f" % (kq, Lx, kq, rec))
                if rec >= TARGET:
                    Lk[kq] = Lx
                    break
            if Lk[kq] is None:
                Lk[kq] = grid[-1]
        Lmax = max(Lk.values())
        # one plan for every launch, tuned on the mix (even odds of the two k)
        mix_big = np.random.default_rng(3).random(nqm) < 0.5
        k_mix = torch.from_numpy(np.where(mix_big, 100, 10).astype(np.int32)).to(dev)
        L_mix = torch.from_numpy(np.where(mix_big, Lk[100], Lk[10]).astype(np.int32)).to(dev)
        splan, _ = ann.ann_autotune_search(base_d, index.graph, qm_d, em, index.medoid, k_mix,
                                           L_mix, 100, Lmax)
        log("serving plan (tuned on the mix): %s" % splan)
        reps = 16
        qs = np.concatenate([qm] * reps)
        truth = np.concatenate([gt100] * reps)
        # the launches of the 4 streams overlap, so as for the pipelined steps
        # the tuned plan is also tried with persistent grids that leave room
        # for the other streams' launches (four-wave workgroups, 16 / 14 / 12
        # wavefronts per CU); the plan with the best saturated throughput on
        # one 160,000-query run serves
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        cands = [splan]
        wq = max(1, int(splan.waves_per_query))
        wpb = 4 if wq == 1 else wq
        for wpc in (16, 14, 12):
            cands.append(ann.make_plan(**dict(splan.as_dict(), waves_per_block=wpb,
                                              blocks=(wpc * cus) // wpb)))
        trials = []
        for cp in cands:
            sv = serve.Server(base_d, index.graph, index.medoid, model=model, slots=4,
                              slot_rows=4096, k_max=100, L_max=Lmax, plan=cp)
            sv.serve(serve.poisson_schedule(qm, 1e12, sizes=(1, 512),
                                            kL=((10, Lk[10]), (100, Lk[100])), seed=7))
            r = sv.serve(serve.poisson_schedule(qs, 1e12, sizes=(1, 512),
                                                kL=((10, Lk[10]), (100, Lk[100])), seed=7))
            trials.append(dict(waves_per_block=int(cp.waves_per_block), blocks=int(cp.blocks),
                               qps=r["qps"]))
            del sv
        splan = cands[max(range(len(cands)), key=lambda i: trials[i]["qps"])]
        log("serving plan: %s (saturated QPS per candidate grid: %s)" %
            (splan, [(t["blocks"], round(t["qps"])) for t in trials]))
        srv = serve.Server(base_d, index.graph, index.medoid, model=model, slots=4,
                           slot_rows=4096, k_max=100, L_max=Lmax, plan=splan)
        out = dict(mix="30% shifted queries, k 10/100", L_by_k=Lk, plan=splan.as_dict(), loads=[],
                   theta=theta, theta_sweep=theta_rows, plan_trials=trials,
                   fallbacks=int((em == index.medoid).sum().item()))
        # capacity: every request waiting at the start (the server saturated);
        # the median of three runs
        srv.serve(serve.poisson_schedule(qm, 1e12, sizes=(1, 512),
                                         kL=((10, Lk[10]), (100, Lk[100])), seed=7))
        sats = [srv.serve(serve.poisson_schedule(qs, 1e12, sizes=(1, 512),
                                                 kL=((10, Lk[10]), (100, Lk[100])), seed=7))
                for _ in range(3)]
        sat = sorted(sats, key=lambda x: x["qps"])[1]
        out["capacity_qps"] = sat["qps"]
        out["capacity_runs_qps"] = [x["qps"] for x in sats]
        log("serving capacity (all requests waiting, median of %s): %s" %
            ([x["qps"] for x in sats], sat))
        for frac in (0.5, 0.8):
            rate = frac * sat["qps"] / 256.5
            sched = serve.poisson_schedule(qs, rate, sizes=(1, 512),
                                           kL=((10, Lk[10]), (100, Lk[100])), seed=7)
            st = srv.serve(sched)
            # served recall@k per request, against the mix's ground truth
            hit = tot = 0
            off = 0
            starts = {}
            for r in sorted(sched, key=lambda r: r.rid):
                starts[r.rid] = off
                off += r.queries.shape[0]
            for r in srv.finished:
                t0 = starts[r.rid]
                tr = truth[t0:t0 + r.queries.shape[0], :r.k]
                hit += int((r.ids[:, :, None] == tr[:, None, :]).any(-1).sum())
                tot += r.ids.size
            st["served_recall"] = round(hit / max(tot, 1), 5)
            # recall@10 of every request (the first 10 ids of k = 100 ones)
            h10 = t10 = 0
            for r in srv.finished:
                t0 = starts[r.rid]
                tr = truth[t0:t0 + r.queries.shape[0], :10]
                h10 += int((r.ids[:, :10, None] == tr[:, None, :]).any(-1).sum())
                t10 += tr.size
            st["served_recall_at_10"] = round(h10 / max(t10, 1), 5)
            st["offered_qps"] = round(frac * sat["qps"], 1)
            out["loads"].append(st)
            log("serving at %.0f%% of capacity: %s" % (100 * frac, st))
        model.c.theta = -float("inf")       # the other legs run without the fallback
        return out

    exacts = {}
    arrays = {}     # per timed leg: the GPU's outputs, exact counts and entries
    med, med_rows, gres, ginfo, abl, g_rows = None, [], None, {}, {}, []
    # ---- medoid entry
    if "medoid" in legs:
        if state is not None:
            L_med, med_rows = int(state["L_medoid"]), state.get("medoid_sweep", [])
            med_hit = bool(state["medoid_reached"])
        else:
            med_rows, L95 = sweep(None, "medoid")
            med_hit = L95 is not None
            L_med = L95 if med_hit else max(med_rows, key=lambda r: r["recall"])["L"]
        med = timed(L_med, None, None, "medoid")
        med["reached_target"] = med_hit
        if state is None and len(targets) > 1:
            med["targets"] = extra_targets(med_rows, None, None, "medoid")

    # ---- GATE entry
    if "gate" in legs:
        tq = None
        if g is None:
            tq = torch.from_numpy(synth.train_queries(w)).to(dev)
            t = time.time()
            gdata = gate.prepare_gate(index, tq, w, n_hubs=args.hubs, log=log)
            g = gate.train_gate(index, gdata, tq, w, hidden=args.hidden, dout=args.dout,
                                epochs=args.epochs, lr=args.lr, tau=args.tau,
                                select_best=args.select_epoch, log=log)
            ginfo = dict(g.info, build_s=round(time.time() - t, 1))
        else:
            ginfo = dict(g.info)
        ent, _, _ = g.select(q_d)
        if state is not None:
            L_gate, g_rows, g_hit = int(state["L_gate"]), state.get("gate_sweep", []), True
        else:
            g_rows, L95 = sweep(ent, "gate")
            g_hit = L95 is not None
            L_gate = L95 if g_hit else max(g_rows, key=lambda r: r["recall"])["L"]
        gres = timed(L_gate, g.model, ent, "gate")
        gres["reached_target"] = g_hit
        gres["sweep"] = g_rows
        if state is None and len(targets) > 1:
            gres["targets"] = extra_targets(g_rows, g.model, ent, "gate")
        if "serve" in legs:
            gres["serving"] = serving(g, L_gate)
        if "ablation" in legs and tq is not None:
            # nearest hub by L2 (no learning) and the untrained towers
            ne = gate.nearest_hub_entries(index, g.hub_ids, q_d)
            n_rows, n_L95 = sweep(ne, "nearest-hub")
            abl["nearest_hub"] = dict(L95=n_L95, sweep=n_rows)
            g0 = gate.train_gate(index, gdata, tq, w, hidden=args.hidden, dout=args.dout,
                                 train=False, log=log)
            e0, _, _ = g0.select(q_d)
            u_rows, u_L95 = sweep(e0, "untrained")
            abl["untrained_towers"] = dict(L95=u_L95, sweep=u_rows)
            del g0
        if "hbkm" in legs and tq is not None:
            # the same entry model on hierarchical balanced k-means hubs
            # (Algorithm 2), against the Lloyd hubs above
            abl["hbkm"] = []
            for lam in [float(x) for x in args.hbkm_lambdas.split(",") if x]:
                gd = gate.prepare_gate(index, tq, w, n_hubs=args.hubs, hubs="hbkm", hbkm_lambda=lam,
                                       log=log)
                gh = gate.train_gate(index, gd, tq, w, hidden=args.hidden, dout=args.dout,
                                     epochs=args.epochs, lr=args.lr, tau=args.tau,
                                     select_best=args.select_epoch, log=log)
                eh, _, _ = gh.select(q_d)
                h_rows, h_L95 = sweep(eh, "hbkm lambda=%g" % lam)
                r95 = next((r for r in h_rows if r["L"] == h_L95), None)
                abl["hbkm"].append(dict(L95=h_L95, ndc=r95["ndc"] if r95 else None,
                                        hubs_s=round(gd.info["hubs_s"], 2), **gd.info["hbkm"],
                                        val_top1=gh.info.get("val_top1"),
                                        val_nearest_hub_top1=gh.info.get("val_nearest_hub_top1")))
                log("hbkm lambda=%g: L95 %s, sizes %d..%d, objective %.3g (Lloyd %.3g)" %
                    (lam, h_L95, gd.info["hbkm"]["size_min"], gd.info["hbkm"]["size_max"],
                     gd.info["hbkm"]["size_objective"], gdata.info.get("size_objective", float("nan"))))
                del gh, gd
        if "fusion" in legs and tq is not None:
            # Eq. 3 fusion embedding in the hub tower's input (the default model is
            # the "without fusion" side)
            gf = gate.train_gate(index, gdata, tq, w, hidden=args.hidden, dout=args.dout,
                                 epochs=args.epochs, lr=args.lr, tau=args.tau, fusion=True, log=log)
            ef, _, _ = gf.select(q_d)
            f_rows, f_L95 = sweep(ef, "fusion")
            r95 = next((r for r in f_rows if r["L"] == f_L95), None)
            abl["fusion"] = dict(L95=f_L95, ndc=r95["ndc"] if r95 else None,
                                 **{k: gf.info.get(k) for k in ("fusion", "train_s", "train_steps",
                                                                 "val_top1", "loss_per_epoch")})
            log("fusion embedding: L95 %s (without fusion %s), held-out agreement %s" %
                (f_L95, L_gate, gf.info.get("val_top1")))
            del gf
        if "queues" in legs and tq is not None:
            # the paper's training signal: Definition 4 queues and Eq. 4 read
            # hub-anchored, on the same hubs, features and towers
            abl["queues"] = []
            for var in [v for v in args.queue_variants.split(",") if v]:
                tp, P, N = [int(x) for x in var.split(":")]
                gq = gate.train_gate(index, gdata, tq, w, hidden=args.hidden, dout=args.dout,
                                     epochs=args.epochs, lr=args.lr, tau=args.tau,
                                     objective="queues", t_pos=tp, queue_P=P, queue_N=N, log=log)
                eq_, _, _ = gq.select(q_d)
                q_rows, q_L95 = sweep(eq_, "queues %s" % var)
                r95 = next((r for r in q_rows if r["L"] == q_L95), None)
                abl["queues"].append(dict(
                    L95=q_L95, ndc=r95["ndc"] if r95 else None, P=P, N=N,
                    **{k: gq.info.get(k) for k in (
                        "queue_hubs_eligible", "queue_pos_mean", "queue_neg_mean", "t_pos", "t_neg",
                        "train_s", "train_steps", "val_top1", "loss_per_epoch")}))
                log("queues objective t_pos=%d P=%d N=%d: L95 %s (labels objective %s)" %
                    (tp, P, N, q_L95, L_gate))
                del gq
        if "nsg" in legs and tq is not None:
            # NSG-style graphs (search-built candidates, alpha = 1) against the
            # kNN + alpha = 1.2 graph above: medoid and GATE entry on each
            abl["nsg"] = []
            keep = index
            deg = lambda gr: round(float((gr >= 0).sum(1).float().mean().item()), 2)  # noqa: E731
            pick = lambda rows, L: next((r for r in rows if r["L"] == L), None)   # noqa: E731
            for Lb in [int(x) for x in args.nsg_L.split(",") if x]:
                nix = gate.build_index_nsg(base_d, knn_k, R, Lb, path=args.nsg_path, log=log)
                log("nsg graph: L_build %d, kNN %d, R %d, medoid %d, bridges %s, %d of %d edges "
                    "from the search pools alone (%.1fs)" %
                    (Lb, knn_k, R, nix.medoid, nix.bridges, nix.edge_stats["from_pool_only"],
                     nix.edge_stats["edges"], nix.build_s))
                index = nix
                m_rows, m_L95 = sweep(None, "nsg%d medoid" % Lb)
                gdn = gate.prepare_gate(index, tq, w, n_hubs=args.hubs, log=log)
                gn = gate.train_gate(index, gdn, tq, w, hidden=args.hidden, dout=args.dout,
                                     epochs=args.epochs, lr=args.lr, tau=args.tau,
                                     select_best=args.select_epoch, log=log)
                en, _, _ = gn.select(q_d)
                n_rows, n_L95 = sweep(en, "nsg%d gate" % Lb)
                n_t = timed(n_L95, gn.model, en, "nsg%d-gate" % Lb) if n_L95 is not None else None
                abl["nsg"].append(dict(
                    L_build=Lb, path=args.nsg_path, build_s=round(nix.build_s, 1),
                    bridges=nix.bridges,
                    degree_mean=deg(nix.graph), **nix.edge_stats,
                    medoid=dict(L95=m_L95, ndc=(pick(m_rows, m_L95) or {}).get("ndc"),
                                best_recall=max(r["recall"] for r in m_rows), sweep=m_rows),
                    gate=dict(L95=n_L95, ndc=(pick(n_rows, n_L95) or {}).get("ndc"), sweep=n_rows,
                              timed={k: n_t[k] for k in (
                                  "qps", "ms_per_step", "search_ms", "recall", "ndc", "hops",
                                  "achieved_gbs", "plan")} if n_t else None)))
                log("nsg graph L_build %d: medoid L95 %s, GATE L95 %s, %s QPS "
                    "(kNN + alpha graph: GATE L95 %s, %s QPS)" %
                    (Lb, m_L95, n_L95, n_t["qps"] if n_t else None, L_gate, gres["qps"]))
                index = keep
                del nix, gdn, gn
            abl["nsg_default_graph"] = dict(
                gate_L95=L_gate, gate_qps=gres["qps"], gate_ndc=gres["ndc"], gate_hops=gres["hops"],
                medoid_L95=med["L"] if med and med["reached_target"] else None,
                degree_mean=deg(keep.graph))
            del keep
        if args.save_state:
            gate.save_state(args.save_state, index, g, dict(
                L_gate=L_gate, L_medoid=med["L"] if med else None,
                medoid_reached=med["reached_target"] if med else None, gate_sweep=g_rows,
                medoid_sweep=med_rows, plan_gate=gres["plan"],
                pipe_plan_gate=gres.get("pipelined", {}).get("plan"),
                plan_medoid=med["plan"] if med else None, exact_gate=exacts.get("gate"),
                exact_medoid=exacts.get("medoid")))
            log("state saved to %s" % args.save_state)
        del tq

    head = gres if (gres is not None and gres["reached_target"]) or med is None else med
    head_label = "gate" if head is gres else "medoid"

    # ---- the highest recall both entries reach, when the medoid never
    # reaches the target: the medoid at its best swept width against GATE at
    # the smallest swept width whose recall reaches that value
    common = None
    if med is not None and gres is not None and not med["reached_target"] and g_rows:
        r_m = med["recall"]
        Lc = next((r["L"] for r in g_rows if r["recall"] >= r_m), None)
        if Lc is not None:
            rc = timed(Lc, g.model, ent, "gate@medoid-best")
            common = dict(recall=r_m, medoid_L=med["L"], medoid_qps=med["qps"], gate_L=Lc,
                          gate_recall=rc["recall"], gate_qps=rc["qps"],
                          gate_over_medoid=round(rc["qps"] / med["qps"], 2))
            log("highest recall both entries reach: %.4f; medoid L=%d %.0f QPS, GATE L=%d "
                "(recall %.4f) %.0f QPS" % (r_m, med["L"], med["qps"], Lc, rc["recall"], rc["qps"]))

    # ---- counter calibration: a plain elementwise kernel that reads and
    # writes COPY_BYTES each
    src_t = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst_t = torch.empty_like(src_t)
    for _ in range(4):
        torch.neg(src_t, out=dst_t)
    torch.cuda.synchronize()
    del src_t, dst_t

    # ---- CPU baseline: the oracle on the same queries, entries and L as the
    # headline; its first pass over the whole batch is also compared with the
    # GPU's results query by query
    cpu = None
    if not args.no_cpu:
        import oracle
        g_host = index.graph.cpu().numpy()
        ga = arrays[head_label]
        ent_host = ga["entry"]
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        cores = min(cores, 16)
        L_cpu = head["L"]
        tot_q, tot_t, first = 0, 0.0, None
        while tot_t < args.cpu_seconds:
            t0 = time.time()
            r = oracle.search(base, g_host, queries, ent_host, k, L_cpu, threads=cores)
            tot_t += time.time() - t0
            tot_q += nq
            first = first or r
        m1 = min(nq, 1000)
        t0 = time.time()
        oracle.search(base, g_host, queries[:m1], ent_host[:m1], k, L_cpu, threads=1)
        t1 = time.time() - t0
        # parity of the timed batch: ids, distances (within 1e-5 relative;
        # exact on integer data), exact distance counts and hops
        rd = first["d2"]
        tol = 1e-5 * np.maximum(rd, 1e-6)
        dist_bad = (np.abs(ga["dist"].astype(np.float64) - rd) > tol).any(1)
        ids_bad = (ga["ids"] != first["ids"]).any(1)
        parity = dict(queries=int(nq), ids_differ=int(ids_bad.sum()),
                      dist_beyond_tol=int(dist_bad.sum()),
                      dist_bitwise_differ=int((ga["dist"].astype(np.float64) != rd).any(1).sum()),
                      ndc_differ=int((ga["ndc"] != first["ndc"]).sum()),
                      hops_differ=int((ga["hops"] != first["hops"]).sum()))
        cpu = dict(value=round(tot_q / tot_t, 2), unit="queries/s", cores=int(cores), kind="oracle",
                   sample="all %d queries x %d passes, %s entries (GPU-selected), L=%d, k=%d, "
                          "FP64 search only" % (nq, tot_q // nq, head_label, L_cpu, k),
                   one_thread=round(m1 / t1, 2), parity_vs_gpu=parity,
                   host=host_cpu()["model"])
        log("cpu oracle: %d queries in %.1fs on %d threads -> %.1f QPS; 1 thread %.1f QPS; "
            "parity over the batch: %s" % (tot_q, tot_t, cores, tot_q / tot_t, m1 / t1, parity))

    achieved = head["achieved_gbs"]
    tr = measured_traffic(args.workload, head["L"], nq, head["plan"]) if head is gres else None
    traffic = None
    if tr is not None:
        traffic = dict(read_bytes=tr[0], write_bytes=tr[1], bytes=tr[0] + tr[1],
                       gbs=round((tr[0] + tr[1]) / (head["search_ms"] / 1000.0) / 1e9, 1))
    workload = ("%s: N=%d d=%d %s, %d queries, %d training queries; graph kNN%d%s/alpha%g/R%d "
                "+ repair; %d hubs; towers %d->%d->%d" %
                (w.name, w.n, w.d, WORKLOAD_TEXT.get(w.name, ""), nq, w.n_train, knn_k,
                 " within %d overlapping groups (x%d)" % (parts, args.overlap) if parts else "",
                 args.alpha, R, args.hubs, w.d, args.hidden, args.dout))
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic["bytes"] if traffic else None)
    summary = dict(
        metric=METRIC, value=head["qps"], unit="queries/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=head["ms_per_step"], higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(
            workload=workload, entry=head_label, k=k, L=head["L"], recall_at_10=head["recall"],
            recall_target=TARGET, reached_target=head["reached_target"],
            ms_per_step_sequential=head.get("ms_per_step_sequential"),
            entry_ms=head["entry_ms"], search_ms=head["search_ms"],
            medoid=dict(reached_target=med["reached_target"], L=med["L"], recall=med["recall"],
                        qps=med["qps"]) if med else None,
            highest_common_recall=common,
            serving=serving_summary(gres.get("serving") if gres else None),
            gate_L_h=(ginfo.get("L_h") if ginfo else None),
            details=args.details or None),
        roofline=roofline,
        cpu_baseline=cpu,
    )
    if args.details:
        full = dict(summary, config=dict(
            summary["config"], workload_text=workload, recall_targets=targets, gate=gres, medoid=med,
            medoid_sweep=med_rows, ablation=abl, gate_build=ginfo,
            graph_build_s=round(index.build_s, 2), bridges=list(index.bridges),
            state=args.load_state or None),
            roofline_detail=dict(roofline, traffic=traffic, kernel="search_kernel",
                                 bytes_per_launch=head["bytes_per_launch"],
                                 launch_ms=head["search_ms"], kernel_hash=search_source_hash()))
        d = os.path.dirname(args.details)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.details, "w") as f:
            json.dump(full, f, indent=1, default=str)
        log("full record written to %s" % args.details)
    line = json.dumps(finite(summary), separators=(",", ":"), allow_nan=False)
    sys.stderr.flush()
    print(line, flush=True)

if __name__ == "__main__":
    main()
