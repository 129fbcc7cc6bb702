"""Continuous-batching request loop over a resident index and entry model.

Requests (a block of query vectors with one k and one L) arrive over time.
The server owns S slots; each slot is a HIP stream with device buffers for up
to `slot_rows` query rows (queries, per-row k and L, entries, results) and
pinned host staging.  Whenever a slot is free, the requests waiting in
arrival order are packed into it while their rows fit, copied in, and the
query path (entry selection, then the persistent search launch, through
ann_query_run) is enqueued on the slot's stream with the results copied back
behind it.  Requests that arrive while others are on the GPU are admitted as
soon as a slot frees, and the slots' work overlaps on the device.  The rows
each slot holds follow from a device-memory budget.

Inside a launch the admitted requests are laid out widest beam first (the
persistent search hands out rows in order), so the longest searches do not
start last and stretch the launch.

Every query's result depends only on its own vector, k, L and entry (one
wavefront per query, per-row tower products), so a request's results are the
same alone and in any mix.
"""
from __future__ import annotations

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


class _Slot:
    def __init__(self, server: "Server", rows: int):
        dev, dim, k_max = server.device, server.dim, server.k_max
        self.rows = rows
        self.stream = torch.cuda.Stream(device=dev)
        self.q = torch.empty((rows, dim), dtype=torch.float32, device=dev)
        self.k = torch.empty(rows, dtype=torch.int32, device=dev)
        self.L = torch.empty(rows, dtype=torch.int32, device=dev)
        self.hq = torch.empty((rows, dim), dtype=torch.float32, pin_memory=True)
        self.hk = torch.empty(rows, dtype=torch.int32, pin_memory=True)
        self.hL = torch.empty(rows, dtype=torch.int32, pin_memory=True)
        self.hids = torch.empty((rows, k_max), dtype=torch.int32, pin_memory=True)
        self.hdist = torch.empty((rows, k_max), dtype=torch.float32, pin_memory=True)
        self.batch = ann.QueryBatch(server.base, server.graph, server.medoid, self.q, self.k,
                                    self.L, k_max, plan=server.plan, model=server.model,
                                    want_stats=False)
        self.event = torch.cuda.Event()
        self.reqs: list[Request] = []
        self.used = 0

    @property
    def busy(self) -> bool:
        return bool(self.reqs)


class Server:
    """S slots over one index (and entry model, or the medoid when None)."""

    def __init__(self, base: torch.Tensor, graph: torch.Tensor, medoid: int,
                 model: ann.EntryModel | None = None, slots: int = 4, slot_rows: int = 0,
                 mem_budget: int = 256 << 20, k_max: int = 100, L_max: int = 256, plan=None,
                 longest_first: bool = True):
        self.base, self.graph, self.medoid, self.model = base, graph, int(medoid), model
        self.longest_first = bool(longest_first)
        self.device = base.device
        n, self.dim = base.shape
        self.k_max = int(k_max)
        self.plan = plan or ann.default_plan(n, self.dim, graph.shape[1], int(L_max))
        self.L_max = int(L_max)
        if self.plan.pool_cap < self.L_max:
            raise ValueError("plan.pool_cap %d < L_max %d" % (self.plan.pool_cap, self.L_max))
        if slot_rows <= 0:
            slot_rows = max(1, mem_budget // (slots * self.bytes_per_row()))
        self.slot_rows = int(slot_rows)
        self.slots = [_Slot(self, self.slot_rows) for _ in range(slots)]
        self.queue: collections.deque[Request] = collections.deque()
        self.finished: list[Request] = []
        self.launches = 0
        self.max_busy = 0
        self.t0 = time.perf_counter()

    def bytes_per_row(self) -> int:
        """Device bytes one admitted query row holds in a slot (entry-stage
        workspace approximated by the tower activations)."""
        b = 4 * self.dim + 4 * 3 + 8 * self.k_max
        if self.model is not None:
            b += 4 * (self.model.qtower.hidden + self.model.qtower.dout) * 2
        return b

    def clock(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        b = req.queries.shape[0]
        if b < 1 or b > self.slot_rows:
            raise ValueError("request %d has %d rows; a slot holds 1..%d" % (req.rid, b,
                                                                           self.slot_rows))
        if not (1 <= req.k <= req.L <= self.L_max and req.k <= self.k_max):
            raise ValueError("request %d: need 1 <= k <= L <= %d and k <= %d" %
                             (req.rid, self.L_max, self.k_max))
        self.queue.append(req)

    def _launch(self, s: _Slot):
        rows = 0
        take = []
        while self.queue and rows + self.queue[0].queries.shape[0] <= s.rows:
            r = self.queue.popleft()
            take.append(r)
            rows += r.queries.shape[0]
        if not rows:
            return
        if self.longest_first:
            # the persistent launch hands out rows in order: the widest
            # searches start first and the short ones fill in behind them
            take.sort(key=lambda r: -r.L)
        rows = 0
        for r in take:
            b = r.queries.shape[0]
            s.hq[rows:rows + b].numpy()[:] = r.queries
            s.hk[rows:rows + b] = r.k
            s.hL[rows:rows + b] = r.L
            s.reqs.append(r)
            rows += b
        s.used = rows
        s.batch.c.nq = rows
        with torch.cuda.stream(s.stream):
            s.q[:rows].copy_(s.hq[:rows], non_blocking=True)
            s.k[:rows].copy_(s.hk[:rows], non_blocking=True)
            s.L[:rows].copy_(s.hL[:rows], non_blocking=True)
            s.batch.run(ann.ANN_STAGE_ALL if self.model is not None else ann.ANN_STAGE_SEARCH,
                        stream=s.stream)
            s.hids[:rows].copy_(s.batch.ids[:rows], non_blocking=True)
            s.hdist[:rows].copy_(s.batch.dist[:rows], non_blocking=True)
            s.event.record(s.stream)
        self.launches += 1

    def _complete(self, s: _Slot):
        now = self.clock()
        off = 0
        for r in s.reqs:
            b = r.queries.shape[0]
            r.ids = s.hids[off:off + b, :r.k].numpy().copy()
            r.dist = s.hdist[off:off + b, :r.k].numpy().copy()
            r.done = now
            off += b
            self.finished.append(r)
        s.reqs = []
        s.used = 0

    def poll(self) -> bool:
        """One pass of the loop: retire finished slots, admit waiting
        requests into free ones.  Returns True when anything happened."""
        acted = False
        for s in self.slots:
            if s.busy and s.event.query():
                self._complete(s)
                acted = True
        for s in self.slots:
            if not self.queue:
                break
            if not s.busy:
                self._launch(s)
                acted = True
        self.max_busy = max(self.max_busy, sum(1 for s in self.slots if s.busy))
        return acted

    def drain(self):
        while self.queue or any(s.busy for s in self.slots):
            if not self.poll():
                time.sleep(20e-6)

    def serve(self, schedule: list[Request]) -> dict:
        """Runs a schedule of requests whose `arrival` times are seconds from
        the start; returns latency and throughput figures."""
        pending = collections.deque(sorted(schedule, key=lambda r: r.arrival))
        self.finished = []
        self.launches = 0
        self.max_busy = 0
        self.t0 = time.perf_counter()
        while pending or self.queue or any(s.busy for s in self.slots):
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
                    mean_ms=round(float(lat.mean()), 3), slots=len(self.slots),
                    slot_rows=self.slot_rows, max_slots_busy=self.max_busy)


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
