"""Streaming service over a device-resident GPMA+ graph.

The paper's framework (Section 3) buffers the edge stream and the queries on
the host, applies update batches to the graph on the GPU and runs ad-hoc and
monitoring queries on it, hiding transfers behind computation.  This module
is the control loop of such a service, MI355X-side:

* continuous batching: whenever the update stream is free, every edge that
  has arrived and is not yet applied (up to `max_batch`) forms the next
  sliding-window step (the same number of oldest edges expire; with
  expire=False the window only grows), applied with fused batching;
* one HBM budget covers all device memory the library holds: the graph
  (array, mirror, the update path's working memory, taken when the service
  starts) and the query slots.  Every allocation of the library goes through
  an allocator that refuses what would pass the budget, and the library then
  returns GPMA_ENOMEM with nothing changed;
* queries (BFS from a vertex, PageRank) are admitted into query slots; a slot
  holds a snapshot of the graph (device copies of the arrays the analytics
  read) plus its scratch; as many slots are made at start as the budget
  leaves room for (up to `max_slots`), each with a snapshot and one run of
  each analytic, so no query pays for an allocation; a query waits in the
  queue until a slot is free;
* an update batch that needs more memory (a root resize grows the array)
  and is refused waits: idle slots are given up, one at a time, until the
  batch fits, waiting for running queries to finish if it must; freed
  budget later lets new slots be made for queued queries;
* an admitted query snapshots the current version on the update stream and
  runs on its slot's own stream, overlapping the updates that follow;
* latency: an edge from its arrival time to the completion of the batch that
  applied it; a query from its arrival time to its result on the host.

All work is done by the HIP library; this is host-side orchestration only.
"""
from __future__ import annotations

import ctypes as C
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from .gpma import (GPMA, GPMA_ENOMEM, GpmaError, TorchAllocator, _check, gpma_bfs, gpma_pagerank,
                   load_library)


@dataclass
class QueryResult:
    qid: int
    kind: str
    arg: int
    version: int
    t_arrival: float
    t_done: float
    result: np.ndarray

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class ServiceReport:
    batches: int = 0
    edges_applied: int = 0          # arrivals taken into the window
    updates_applied: int = 0        # inserts + deletes that changed the graph
    duration_s: float = 0.0
    edge_latency_s: List[float] = field(default_factory=list)
    queries: List[QueryResult] = field(default_factory=list)
    slots: int = 0
    max_queue: int = 0
    batch_sizes: List[int] = field(default_factory=list)
    update_waits: int = 0           # batches refused for memory, applied after slots gave way
    slots_given_up: int = 0
    slots_made: int = 0             # slots made during the run (budget freed)
    budget_bytes: int = 0
    peak_bytes: int = 0
    t_last_update: float = 0.0      # when the last step completed (from the start of the run)

    @staticmethod
    def _pct(xs, q):
        if len(xs) == 0:
            return None
        return float(np.percentile(np.asarray(xs), q))

    def summary(self) -> dict:
        ql = [q.latency for q in self.queries]
        return {
            "batches": self.batches,
            "edges_applied": self.edges_applied,
            "updates_applied": self.updates_applied,
            "updates_per_s": (self.updates_applied / self.duration_s) if self.duration_s else None,
            "updates_per_s_until_last_step": (self.updates_applied / self.t_last_update)
            if self.t_last_update else None,
            "edges": len(self.edge_latency_s),
            "edge_latency_ms_p50": None if not self.edge_latency_s else 1e3 * self._pct(self.edge_latency_s, 50),
            "edge_latency_ms_p99": None if not self.edge_latency_s else 1e3 * self._pct(self.edge_latency_s, 99),
            "queries": len(self.queries),
            "query_latency_ms_p50": None if not ql else 1e3 * self._pct(ql, 50),
            "query_latency_ms_p99": None if not ql else 1e3 * self._pct(ql, 99),
            "query_slots": self.slots,
            "max_query_queue": self.max_queue,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "update_waits": self.update_waits,
            "slots_given_up": self.slots_given_up,
            "slots_made": self.slots_made,
            "budget_bytes": self.budget_bytes,
            "peak_bytes": self.peak_bytes,
        }


class BudgetAllocator(TorchAllocator):
    """torch's caching allocator under an HBM budget: a request that would
    take the bytes held through this allocator past `budget` is refused."""

    def __init__(self, budget: int):
        super().__init__()
        self.budget = int(budget)

    def allow(self, nbytes: int) -> bool:
        return self.held_bytes + nbytes <= self.budget


class _Slot:
    """One admitted-query slot: a snapshot handle, its stream and vectors."""

    def __init__(self, V: int):
        self.V = V
        self.snap = None
        self.cap = 0          # capacity the slot's scratch was taken for
        self.stream = torch.cuda.Stream()
        self.dist = torch.empty(V, dtype=torch.int32, device="cuda")
        self.x = torch.empty(V, dtype=torch.float32, device="cuda")

    def close(self):
        if self.snap is not None:
            load_library().gpma_destroy(self.snap)
            self.snap = None


class GraphService:
    def __init__(self, V: int, window: torch.Tensor, leaf_size: int = 0, mirror: bool = True,
                 hbm_budget_bytes: Optional[int] = None, max_batch: int = 1 << 16,
                 pr_iters: int = 10, max_slots: int = 4, expire: bool = True):
        self._lib = load_library()
        self.V = V
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget_bytes = free // 4
        self.alloc = BudgetAllocator(hbm_budget_bytes)
        self.g = GPMA(V, window, leaf_size=leaf_size, mirror=mirror, allocator=self.alloc)
        # the update path's working memory for steps of up to max_batch
        # arrivals (a step deletes and inserts that many, fused)
        self.g.reserve(2 * max_batch)
        # the live window in arrival order (oldest first), then the arrivals of
        # the current run: order[head:tail] are live, order[tail:] still to come
        self.order = window
        self.head = 0
        self.tail = window.numel()
        self.max_batch = max_batch
        self.pr_iters = pr_iters
        self.expire = expire
        self.max_slots = max_slots
        self.ustream = torch.cuda.Stream()
        self.slot_bytes = 0                 # device bytes a slot took when it was made
        self.slots: List[Optional[_Slot]] = []
        while len(self.slots) < max_slots and self._make_slot():
            pass
        if not self.slots:
            self.close()
            raise ValueError("the HBM budget leaves no room for a query slot")
        self.version = 0
        self.record = False
        self.batch_log = []                 # (deleted, inserted) per version step, on host, if record

    def close(self):
        for s in self.slots:
            if s is not None:
                s.close()
        self.slots = []
        self.g.close()

    # ---- slots under the budget
    def _make_slot(self) -> bool:
        """A new slot; False, with nothing kept, when the budget refuses."""
        if self.slot_bytes and self.alloc.held_bytes + self.slot_bytes > self.alloc.budget:
            return False
        held = self.alloc.held_bytes
        slot = _Slot(self.V)
        if self._prepare(slot) is None:
            return False
        self.slot_bytes = max(self.slot_bytes, self.alloc.held_bytes - held)
        self.slots.append(slot)
        return True

    def _prepare(self, slot: _Slot):
        """Snapshot the current version into the slot and, when the array's
        capacity changed since the slot last ran, one run of each analytic to
        take their scratch now; the event that orders the snapshot, or None
        (the slot's memory released) when the budget refuses."""
        try:
            ev = self._snapshot_into(slot)
            if slot.cap != self.g.capacity:
                self.ustream.synchronize()
                gpma_pagerank(slot.snap, None, slot.x, 1, 0.85, stream=slot.stream)
                gpma_bfs(slot.snap, 0, slot.dist, stream=slot.stream)
                slot.stream.synchronize()
                slot.cap = self.g.capacity
            return ev
        except GpmaError as e:
            slot.close()
            if e.code != GPMA_ENOMEM:
                raise
            return None

    # ---- one sliding-window step on the update stream: the k oldest edges
    # expire (unless the window only grows), the k arrivals
    # order[tail:tail+k] enter (Section 3: a sliding window over the edge
    # stream); returns the step's summed statistics
    def _apply(self, k: int):
        dels = self.order[self.head:self.head + k] if self.expire else self.order[:0]
        ins = self.order[self.tail:self.tail + k]
        assert ins.numel() == k, "arrivals past the end of the stream"
        with torch.cuda.stream(self.ustream):
            st = self.g.apply_batches([1, 0], [dels, ins], stream=self.ustream)
        if self.expire:
            self.head += k
        self.tail += k
        self.version += 1
        if self.record:
            self.batch_log.append((dels.cpu(), ins.cpu()))
        return st

    # ---- a query on a slot
    def _snapshot_into(self, slot: _Slot):
        if slot.snap is None:
            h = C.c_void_p()
            _check(self._lib.gpma_snapshot(self.g.h, C.byref(h), C.c_void_p(self.ustream.cuda_stream)),
                   "gpma_snapshot")
            slot.snap = h
        else:
            _check(self._lib.gpma_snapshot_refresh(self.g.h, slot.snap, C.c_void_p(self.ustream.cuda_stream)),
                   "gpma_snapshot_refresh")
        ev = torch.cuda.Event()
        ev.record(self.ustream)
        return ev

    def _run_query(self, slot: _Slot, ev, qid, kind, arg, t_arr, t0, version) -> QueryResult:
        slot.stream.wait_event(ev)
        if kind == "bfs":
            gpma_bfs(slot.snap, int(arg), slot.dist, stream=slot.stream)
            res = slot.dist.to("cpu", non_blocking=False)
        else:
            gpma_pagerank(slot.snap, None, slot.x, int(arg) or self.pr_iters, 0.85, stream=slot.stream)
            slot.stream.synchronize()
            res = slot.x.cpu()
        slot.stream.synchronize()
        return QueryResult(qid, kind, int(arg), version, t_arr, time.perf_counter() - t0, res.numpy())

    # ---- the loop
    def run(self, edge_times: torch.Tensor, edges: torch.Tensor, query_times, query_kinds, query_args,
            time_limit_s: float = 10.0) -> ServiceReport:
        """edge_times (seconds, ascending, host float64 tensor) and edges (device
        keys, same length); queries: parallel host lists.  Runs until every
        edge is applied and every query answered (or the time limit)."""
        rep = ServiceReport(slots=sum(1 for s in self.slots if s is not None), budget_bytes=self.alloc.budget)
        # arrival order from here on: the live window, then this run's edges
        self.order = torch.cat([self.order[self.head:self.tail], edges.to(self.order.device)])
        self.tail -= self.head
        self.head = 0
        et = edge_times.numpy()
        ne = len(et)
        nq = len(query_times)
        applied_to = 0
        released_q = 0
        queue: List[int] = []
        free = [i for i, s in enumerate(self.slots) if s is not None]     # idle slots
        running = {}
        pool = ThreadPoolExecutor(max_workers=self.max_slots)
        t0 = time.perf_counter()

        def reap(block: bool):
            """Completed queries give their slots back (block: wait for one)."""
            if block and running:
                next(iter(running.values()))[0].result()
            for qi in [q for q, (f, si) in running.items() if f.done()]:
                f, si = running.pop(qi)
                rep.queries.append(f.result())
                free.append(si)

        def give_up_slot() -> bool:
            """Release an idle slot's memory (waiting for a query to finish if
            every slot is busy); False when no slot is left to give up."""
            if not free:
                if not running:
                    return False
                reap(True)
            si = free.pop()
            self.slots[si].close()
            self.slots[si] = None
            rep.slots_given_up += 1
            return True

        while True:
            now = time.perf_counter() - t0
            if now > time_limit_s:
                break
            # queries that arrived join the queue
            while released_q < nq and query_times[released_q] <= now:
                queue.append(released_q)
                released_q += 1
            rep.max_queue = max(rep.max_queue, len(queue))
            reap(False)
            # a queue and budget to spare: a slot in place of one given up
            live = sum(1 for s in self.slots if s is not None)
            if queue and not free and live < self.max_slots and self._make_slot():
                free.append(len(self.slots) - 1)
                rep.slots_made += 1
            # admit queued queries while slots allow: snapshot now
            while queue and free:
                si = free.pop()
                ev = self._prepare(self.slots[si])
                if ev is None:          # the array grew past what this slot may hold
                    self.slots[si] = None
                    rep.slots_given_up += 1
                    continue
                qi = queue.pop(0)
                fut = pool.submit(self._run_query, self.slots[si], ev, qi, query_kinds[qi], query_args[qi],
                                  float(query_times[qi]), t0, self.version)
                running[qi] = (fut, si)
            # continuous batching: everything that has arrived, up to max_batch
            hi = int(np.searchsorted(et, now, side="right"))
            hi = min(hi, applied_to + self.max_batch)
            if hi > applied_to:
                waited = False
                while True:
                    try:
                        st = self._apply(hi - applied_to)
                        break
                    except GpmaError as e:      # nothing changed: make room, then again
                        if e.code != GPMA_ENOMEM or not give_up_slot():
                            raise
                        waited = True
                rep.update_waits += int(waited)
                done_t = time.perf_counter() - t0
                rep.t_last_update = done_t
                rep.edge_latency_s.extend((done_t - et[applied_to:hi]).tolist())
                rep.batches += 1
                rep.edges_applied += hi - applied_to
                rep.updates_applied += st.applied
                rep.batch_sizes.append(hi - applied_to)
                applied_to = hi
            elif applied_to >= ne and released_q >= nq and not queue and not running:
                break
            else:
                nxt = []
                if applied_to < ne:
                    nxt.append(et[applied_to])
                if released_q < nq:
                    nxt.append(query_times[released_q])
                if nxt and not running and not queue:
                    wait = min(nxt) - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                elif queue and not free and running:
                    reap(True)
        for qi, (f, si) in running.items():
            rep.queries.append(f.result())
        pool.shutdown(wait=True)
        rep.duration_s = time.perf_counter() - t0
        rep.peak_bytes = self.alloc.peak_bytes
        return rep
