"""Streaming service over a device-resident GPMA+ graph.

The paper's framework (Section 3) buffers the edge stream and the queries on
the host, applies update batches to the graph on the GPU and runs ad-hoc and
monitoring queries on it, hiding transfers behind computation.  This module
is the control loop of such a service, MI355X-side:

* continuous batching: whenever the update stream is free, every edge that
  has arrived and is not yet applied (up to `max_batch`) forms the next
  sliding-window step (the same number of oldest edges expire), applied with
  fused batching;
* queries (BFS from a vertex, PageRank) are admitted into query slots; a slot
  holds a snapshot of the graph (device copies of the arrays the analytics
  read) plus its scratch, so the number of slots is the HBM budget divided
  by the bytes of one slot; a query waits in the queue until a slot is free;
  every slot takes its memory when the service starts (a snapshot and one
  run of each analytic), so no query pays for an allocation;
* an admitted query snapshots the current version on the update stream and
  runs on its slot's own stream, overlapping the updates that follow;
* latency: an edge from its arrival time to the completion of the batch that
  applied it; a query from its arrival time to its result on the host.

All work is done by the HIP library; this is host-side orchestration only.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from .gpma import GPMA, _check, _HandleView, gpma_bfs, gpma_pagerank, load_library


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
            "edge_latency_ms_p50": None if not self.edge_latency_s else 1e3 * self._pct(self.edge_latency_s, 50),
            "edge_latency_ms_p99": None if not self.edge_latency_s else 1e3 * self._pct(self.edge_latency_s, 99),
            "queries": len(self.queries),
            "query_latency_ms_p50": None if not ql else 1e3 * self._pct(ql, 50),
            "query_latency_ms_p99": None if not ql else 1e3 * self._pct(ql, 99),
            "query_slots": self.slots,
            "max_query_queue": self.max_queue,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
        }


class _Slot:
    """One admitted-query slot: a snapshot handle, its stream and scratch."""

    def __init__(self, V: int):
        self.V = V
        self.snap = None
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
                 pr_iters: int = 10, max_slots: int = 4):
        self._lib = load_library()
        self.V = V
        self.g = GPMA(V, window, leaf_size=leaf_size, mirror=mirror)
        # the live window in arrival order (oldest first), then the arrivals of
        # the current run: order[head:tail] are live, order[tail:] still to come
        self.order = window
        self.head = 0
        self.tail = window.numel()
        self.max_batch = max_batch
        self.pr_iters = pr_iters
        self.ustream = torch.cuda.Stream()
        # a slot: the snapshot (array and mirror), PageRank's scratch (packed
        # edges, 8 B a slot of the array; binned records, 10 B an entry; fp64
        # vectors), BFS queues and the slot's own vectors
        cap, n_ent = int(self.g.capacity), int(self.g.num_edges) + V
        slot_bytes = (int(self._lib.gpma_device_bytes(self.g.h)) + 8 * cap + 10 * n_ent
                      + V * (4 + 4 + 8 + 8 + 4 + 4 + 4))
        self.slot_bytes = slot_bytes
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget_bytes = free // 4
        n = int(max(1, min(max_slots, hbm_budget_bytes // slot_bytes)))
        self.slots = [_Slot(V) for _ in range(n)]
        for slot in self.slots:   # reserve every slot's memory now
            self._snapshot_into(slot)
            self.ustream.synchronize()
            gpma_pagerank(slot.snap, None, slot.x, 1, 0.85, stream=slot.stream)
            gpma_bfs(slot.snap, 0, slot.dist, stream=slot.stream)
            slot.stream.synchronize()
        self.version = 0
        self.record = False
        self.batch_log = []                 # (deleted, inserted) per version step, on host, if record

    def close(self):
        for s in self.slots:
            s.close()
        self.g.close()

    # ---- one sliding-window step on the update stream: the k oldest edges
    # expire, the k arrivals order[tail:tail+k] enter (Section 3: a sliding
    # window over the edge stream); returns the step's summed statistics
    def _apply(self, k: int):
        dels = self.order[self.head:self.head + k]
        ins = self.order[self.tail:self.tail + k]
        assert ins.numel() == k, "arrivals past the end of the stream"
        with torch.cuda.stream(self.ustream):
            st = self.g.apply_batches([1, 0], [dels, ins], stream=self.ustream)
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
        rep = ServiceReport(slots=len(self.slots))
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
        free = list(range(len(self.slots)))
        running = {}
        pool = ThreadPoolExecutor(max_workers=len(self.slots))
        lock = threading.Lock()
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            if now > time_limit_s:
                break
            # queries that arrived join the queue
            while released_q < nq and query_times[released_q] <= now:
                queue.append(released_q)
                released_q += 1
            rep.max_queue = max(rep.max_queue, len(queue))
            # completed queries free their slots
            for qi in [q for q, (f, si) in running.items() if f.done()]:
                f, si = running.pop(qi)
                rep.queries.append(f.result())
                free.append(si)
            # admit queued queries while slots (HBM budget) allow: snapshot now
            while queue and free:
                qi = queue.pop(0)
                si = free.pop()
                ev = self._snapshot_into(self.slots[si])
                fut = pool.submit(self._run_query, self.slots[si], ev, qi, query_kinds[qi], query_args[qi],
                                  float(query_times[qi]), t0, self.version)
                running[qi] = (fut, si)
            # continuous batching: everything that has arrived, up to max_batch
            hi = int(np.searchsorted(et, now, side="right"))
            hi = min(hi, applied_to + self.max_batch)
            if hi > applied_to:
                st = self._apply(hi - applied_to)
                done_t = time.perf_counter() - t0
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
        for qi, (f, si) in running.items():
            rep.queries.append(f.result())
        pool.shutdown(wait=True)
        rep.duration_s = time.perf_counter() - t0
        return rep
