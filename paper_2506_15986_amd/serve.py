"""Continuous-batching request loop over a resident index and entry model.

Requests (a block of query vectors with one k and one L) arrive over time.
Admission is by memory, row by row: the server owns one pool of query rows on
the device (queries, per-row k and L, entries, results) with pinned host
staging, sized from a device-memory budget, and S launch streams.  Whenever a
stream is free and the requests waiting in arrival order fit in a free range
of the pool (first fit, at most `launch_rows` rows per launch), they take
exactly the rows they need, are copied in, and the query path (entry
selection, then the persistent search launch, through ann_query_run) is
enqueued on the stream with the results copied back behind it.  When a
launch completes its rows return to the pool at once, so a one-query request
holds one row, and requests that arrive while others are on the GPU are
admitted as streams and rows free up; the launches overlap on the device.

Inside a launch the admitted requests are laid out widest beam first (the
persistent search hands out rows in order), so the longest searches do not
start last and stretch the launch.

Every query's result depends only on its own vector, k, L and entry (one
wavefront per query, per-row tower products), so a request's results are the
same alone and in any mix.
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import time

import numpy as np
import torch

from . import ann


@dataclasses.dataclass
class Request:
    rid: int
    queries: np.ndarray          # [b, dim] float32
    k: int
    L: int
    arrival: float = 0.0         # seconds on the server's clock
    done: float = -1.0
    ids: np.ndarray | None = None
    dist: np.ndarray | None = None


class RowPool:
    """First-fit allocator of contiguous row ranges in [0, rows)."""

    def __init__(self, rows: int):
        self.rows = int(rows)
        self.free = [(0, self.rows)]          # (start, length), sorted, never adjacent

    def largest(self) -> int:
        return max((ln for _, ln in self.free), default=0)

    def alloc(self, n: int) -> int:
        for t, (st, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[t]
                else:
                    self.free[t] = (st + n, ln - n)
                return st
        return -1

    def release(self, st: int, n: int):
        t = bisect.bisect_left(self.free, (st, 0))
        self.free.insert(t, (st, n))
        # merge with the neighbours
        if t + 1 < len(self.free) and st + n == self.free[t + 1][0]:
            self.free[t] = (st, n + self.free[t + 1][1])
            del self.free[t + 1]
        if t > 0 and self.free[t - 1][0] + self.free[t - 1][1] == st:
            self.free[t - 1] = (self.free[t - 1][0], self.free[t - 1][1] + self.free[t][1])
            del self.free[t]

    def in_use(self) -> int:
        return self.rows - sum(ln for _, ln in self.free)


class _Stream:
    """One launch stream: its workspaces (sized for launch_rows) and the
    requests of its launch in flight."""

    def __init__(self, server: "Server"):
        sv = server
        # a hardware queue of its own, so that the slots' launches overlap
        self.stream = ann.dedicated_stream(len(sv.streams_made), sv.device)
        sv.streams_made.append(self)
        m = sv.launch_rows
        self.batch = ann.QueryBatch(sv.base, sv.graph, sv.medoid, sv.q[:m], sv.k[:m], sv.L[:m],
                                    sv.k_max, plan=sv.plan, model=sv.model,
                                    entry_ids=sv.entry[:m] if sv.model is not None else None,
                                    want_stats=False)
        self.event = torch.cuda.Event()
        self.reqs: list[Request] = []
        self.off = 0
        self.used = 0

    @property
    def busy(self) -> bool:
        return bool(self.reqs)


class Server:
    """A pool of query rows and S launch streams over one index (and entry
    model, or the medoid when None).

    slots       launch streams (launches in flight at once)
    slot_rows   the most rows one launch takes (default: the whole pool)
    pool_rows   rows of the shared pool (default: slots * slot_rows when
                slot_rows is given, else what mem_budget buys)"""

    def __init__(self, base: torch.Tensor, graph: torch.Tensor, medoid: int,
                 model: ann.EntryModel | None = None, slots: int = 4, slot_rows: int = 0,
                 mem_budget: int = 256 << 20, k_max: int = 100, L_max: int = 256, plan=None,
                 longest_first: bool = True, pool_rows: int = 0):
        self.base, self.graph, self.medoid, self.model = base, graph, int(medoid), model
        self.longest_first = bool(longest_first)
        self.device = dev = base.device
        n, self.dim = base.shape
        self.k_max = int(k_max)
        self.plan = plan or ann.default_plan(n, self.dim, graph.shape[1], int(L_max))
        self.L_max = int(L_max)
        if self.plan.pool_cap < self.L_max:
            raise ValueError("plan.pool_cap %d < L_max %d" % (self.plan.pool_cap, self.L_max))
        if pool_rows <= 0:
            pool_rows = slots * slot_rows if slot_rows > 0 else \
                max(1, mem_budget // self.bytes_per_row())
        self.pool_rows = int(pool_rows)
        self.launch_rows = int(min(slot_rows, pool_rows)) if slot_rows > 0 else self.pool_rows
        P, dim = self.pool_rows, self.dim
        self.q = torch.empty((P, dim), dtype=torch.float32, device=dev)
        self.k = torch.empty(P, dtype=torch.int32, device=dev)
        self.L = torch.empty(P, dtype=torch.int32, device=dev)
        self.entry = torch.empty(P, dtype=torch.int32, device=dev)
        self.ids = torch.empty((P, self.k_max), dtype=torch.int32, device=dev)
        self.dist = torch.empty((P, self.k_max), dtype=torch.float32, device=dev)
        self.hq = torch.empty((P, dim), dtype=torch.float32, pin_memory=True)
        self.hk = torch.empty(P, dtype=torch.int32, pin_memory=True)
        self.hL = torch.empty(P, dtype=torch.int32, pin_memory=True)
        self.hids = torch.empty((P, self.k_max), dtype=torch.int32, pin_memory=True)
        self.hdist = torch.empty((P, self.k_max), dtype=torch.float32, pin_memory=True)
        self.pool = RowPool(P)
        self.streams_made: list = []
        self.streams = [_Stream(self) for _ in range(slots)]
        self.slot_rows = self.launch_rows
        self.queue: collections.deque[Request] = collections.deque()
        self.finished: list[Request] = []
        self.launches = 0
        self.max_busy = 0
        self.max_rows = 0
        self.t0 = time.perf_counter()

    def bytes_per_row(self) -> int:
        """Device bytes one admitted query row holds in the pool (entry-stage
        workspace approximated by the tower activations)."""
        b = 4 * self.dim + 4 * 4 + 8 * self.k_max
        if self.model is not None:
            b += 4 * (self.model.qtower.hidden + self.model.qtower.dout) * 2
        return b

    def clock(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        b = req.queries.shape[0]
        if b < 1 or b > self.launch_rows:
            raise ValueError("request %d has %d rows; a launch holds 1..%d" % (req.rid, b,
                                                                             self.launch_rows))
        if not (1 <= req.k <= req.L <= self.L_max and req.k <= self.k_max):
            raise ValueError("request %d: need 1 <= k <= L <= %d and k <= %d" %
                             (req.rid, self.L_max, self.k_max))
        self.queue.append(req)

    def _launch(self, s: _Stream) -> bool:
        """Admits the waiting requests (arrival order) that fit in the largest
        free range of the pool, up to launch_rows, onto stream s."""
        room = min(self.pool.largest(), self.launch_rows)
        rows = 0
        take = []
        while self.queue and rows + self.queue[0].queries.shape[0] <= room:
            r = self.queue.popleft()
            take.append(r)
            rows += r.queries.shape[0]
        if not rows:
            return False
        off = self.pool.alloc(rows)
        assert off >= 0
        if self.longest_first:
            # the persistent launch hands out rows in order: the widest
            # searches start first and the short ones fill in behind them
            take.sort(key=lambda r: -r.L)
        o = off
        for r in take:
            b = r.queries.shape[0]
            self.hq[o:o + b].numpy()[:] = r.queries
            self.hk[o:o + b] = r.k
            self.hL[o:o + b] = r.L
            s.reqs.append(r)
            o += b
        s.off, s.used = off, rows
        e = slice(off, off + rows)
        s.batch.rebind(self.q[e], self.k[e], self.L[e],
                       self.entry[e] if self.model is not None else None, self.ids[e],
                       self.dist[e])
        with torch.cuda.stream(s.stream):
            self.q[e].copy_(self.hq[e], non_blocking=True)
            self.k[e].copy_(self.hk[e], non_blocking=True)
            self.L[e].copy_(self.hL[e], non_blocking=True)
            s.batch.run(ann.ANN_STAGE_ALL if self.model is not None else ann.ANN_STAGE_SEARCH,
                        stream=s.stream)
            self.hids[e].copy_(self.ids[e], non_blocking=True)
            self.hdist[e].copy_(self.dist[e], non_blocking=True)
            s.event.record(s.stream)
        self.launches += 1
        return True

    def _complete(self, s: _Stream):
        now = self.clock()
        off = s.off
        for r in s.reqs:
            b = r.queries.shape[0]
            r.ids = self.hids[off:off + b, :r.k].numpy().copy()
            r.dist = self.hdist[off:off + b, :r.k].numpy().copy()
            r.done = now
            off += b
            self.finished.append(r)
        self.pool.release(s.off, s.used)
        s.reqs = []
        s.used = 0

    def poll(self) -> bool:
        """One pass of the loop: retire finished launches (their rows return
        to the pool), admit waiting requests onto free streams while rows fit.
        Returns True when anything happened."""
        acted = False
        for s in self.streams:
            if s.busy and s.event.query():
                self._complete(s)
                acted = True
        for s in self.streams:
            if not self.queue:
                break
            if not s.busy and self._launch(s):
                acted = True
        self.max_busy = max(self.max_busy, sum(1 for s in self.streams if s.busy))
        self.max_rows = max(self.max_rows, self.pool.in_use())
        return acted

    def drain(self):
        while self.queue or any(s.busy for s in self.streams):
            if not self.poll():
                time.sleep(20e-6)

    def serve(self, schedule: list[Request]) -> dict:
        """Runs a schedule of requests whose `arrival` times are seconds from
        the start; returns latency and throughput figures."""
        pending = collections.deque(sorted(schedule, key=lambda r: r.arrival))
        self.finished = []
        self.launches = 0
        self.max_busy = 0
        self.max_rows = 0
        self.t0 = time.perf_counter()
        while pending or self.queue or any(s.busy for s in self.streams):
            now = self.clock()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if not self.poll():
                time.sleep(20e-6)
        wall = self.clock()
        lat = np.array([r.done - r.arrival for r in self.finished]) * 1000.0
        nq = sum(r.queries.shape[0] for r in self.finished)
        return dict(requests=len(self.finished), queries=nq, wall_s=round(wall, 4),
                    qps=round(nq / wall, 1), launches=self.launches,
                    p50_ms=round(float(np.percentile(lat, 50)), 3),
                    p99_ms=round(float(np.percentile(lat, 99)), 3),
                    mean_ms=round(float(lat.mean()), 3), streams=len(self.streams),
                    pool_rows=self.pool_rows, launch_rows=self.launch_rows,
                    max_slots_busy=self.max_busy, max_rows_in_use=self.max_rows)


def poisson_schedule(queries: np.ndarray, rate_per_s: float, sizes=(1, 512), kL=((10, 64),),
                     seed: int = 0) -> list[Request]:
    """Requests cut from `queries` in order: sizes uniform on [sizes], (k, L)
    drawn uniformly from kL, exponential inter-arrival gaps at the rate."""
    rng = np.random.default_rng(seed)
    out, i, t, rid = [], 0, 0.0, 0
    while i < queries.shape[0]:
        b = int(min(rng.integers(sizes[0], sizes[1] + 1), queries.shape[0] - i))
        k, L = kL[int(rng.integers(0, len(kL)))]
        out.append(Request(rid, np.ascontiguousarray(queries[i:i + b]), int(k), int(L), t))
        i += b
        rid += 1
        t += float(rng.exponential(1.0 / rate_per_s))
    return out
