"""Continuous-batching request loop over resident indexes.

Requests (an index name, a block of queries, a radius) arrive at any time.
One scheduler thread keeps up to `streams` batches in flight on the GPU:
whenever a stream slot is free it packs the oldest waiting requests of one
index -- any mix of radii, each query keeping its own -- into one batch of at
most `max_batch` queries, admitted only while the queries in flight stay
within the memory budget, and enqueues the library's synchronisation-free
batched path (fclsh_query_batch_async) on that slot's stream.  Batches on
different streams overlap on the device; a finished batch (its event has
fired) is split back into its requests, whose futures complete with their
neighbour lists.  Latency = completion time - submit time.

All compute runs in the HIP library; this module only schedules and moves
bytes.  Every answer equals the answer of the same request sent alone,
because queries of a batch never interact.
"""
from __future__ import annotations

import collections
import concurrent.futures
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import Index, QUERY_IDS_OVERFLOW, QUERY_PAIR_OVERFLOW, QUERY_SPILL_OVERFLOW, words


@dataclass
class Request:
    index: str
    queries: np.ndarray  # uint64 [m, W]
    radius: int
    t_submit: float
    future: concurrent.futures.Future = field(default_factory=concurrent.futures.Future)
    t_done: float = 0.0


@dataclass
class _Slot:
    stream: object
    qbuf: object
    rbuf: object
    offsets: object
    ids: object
    result: object
    host_q: object
    host_r: object
    event: object = None
    batch: list = None
    index: str = ""
    nq: int = 0


class Server:
    """Serve exact r-NN requests against resident indexes.

    indexes        name -> built Index (kept resident in HBM)
    max_batch      queries per launched batch (also the per-slot capacity)
    streams        batches in flight at once (one HIP stream each)
    mem_budget     bytes of per-batch device state allowed in flight; a request
                   waits while admitting it would exceed it
    ids_per_query  result capacity per query of a slot; a batch that does not
                   fit is rerun synchronously with exact sizing
    """

    def __init__(self, indexes: dict, max_batch: int = 4096, streams: int = 3,
                 mem_budget: int = 8 << 30, ids_per_query: int = 64):
        import torch

        self.torch = torch
        self.indexes = dict(indexes)
        self.max_batch = int(max_batch)
        self.mem_budget = int(mem_budget)
        self.lock = threading.Lock()
        self.pending = collections.deque()
        self.stop_flag = False
        self.latencies = []
        self.completed = 0
        self.queries_done = 0
        self.bytes_in_flight = 0
        self.batches = 0
        wmax = max(words(ix.d) for ix in self.indexes.values())
        cap = self.max_batch * ids_per_query
        self.slots = []
        for _ in range(streams):
            st = torch.cuda.Stream()
            slot = _Slot(
                stream=st,
                qbuf=torch.empty((self.max_batch, wmax), dtype=torch.int64, device="cuda"),
                rbuf=torch.empty(self.max_batch, dtype=torch.int32, device="cuda"),
                offsets=torch.empty(self.max_batch + 1, dtype=torch.int64, device="cuda"),
                ids=torch.empty(cap, dtype=torch.int32, device="cuda"),
                result=torch.zeros(2, dtype=torch.int64, device="cuda"),
                host_q=torch.empty((self.max_batch, wmax), dtype=torch.int64, pin_memory=True),
                host_r=torch.empty(self.max_batch, dtype=torch.int32, pin_memory=True),
            )
            for ix in self.indexes.values():
                ix.reserve(self.max_batch, pair_capacity=cap, spill_capacity=1 << 18, stream=st)
            self.slots.append(slot)
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # ------------------------------------------------------------------ API
    def submit(self, index: str, queries: np.ndarray, radius: int) -> concurrent.futures.Future:
        if index not in self.indexes:
            raise KeyError(index)
        ix = self.indexes[index]
        q = np.ascontiguousarray(queries, np.uint64)
        if q.ndim != 2 or q.shape[1] != words(ix.d):
            raise ValueError("queries must be uint64 [m, W]")
        if q.shape[0] > self.max_batch:
            raise ValueError("a request may hold at most max_batch queries")
        if not 0 <= radius <= ix.info["r"]:
            raise ValueError("radius outside [0, index radius]")
        req = Request(index, q, int(radius), time.perf_counter())
        with self.lock:
            self.pending.append(req)
        return req.future

    def close(self):
        self.stop_flag = True
        self.thread.join()

    def stats(self) -> dict:
        lat = np.asarray(self.latencies, np.float64)
        return {"requests": self.completed, "queries": self.queries_done, "batches": self.batches,
                "p50_ms": float(np.percentile(lat, 50)) * 1e3 if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99)) * 1e3 if lat.size else None,
                "mean_ms": float(lat.mean()) * 1e3 if lat.size else None}

    # ------------------------------------------------------------ internals
    def _batch_bytes(self, ix: Index, nq: int) -> int:
        L = ix.info["L"]
        return nq * (words(ix.d) * 8 + 4 + L * 16 + 16 + 64 * 4)

    def _form_batch(self):
        """Oldest waiting requests of the oldest request's index, within
        max_batch queries and the memory budget."""
        with self.lock:
            if not self.pending:
                return None, [], 0
            name = self.pending[0].index
            ix = self.indexes[name]
            take, nq, keep = [], 0, collections.deque()
            while self.pending:
                r = self.pending.popleft()
                m = r.queries.shape[0]
                fits = r.index == name and nq + m <= self.max_batch and (
                    self.bytes_in_flight + self._batch_bytes(ix, nq + m) <= self.mem_budget
                    or (not take and self.bytes_in_flight == 0))  # a lone request always runs
                if fits:
                    take.append(r)
                    nq += m
                else:
                    keep.append(r)
                    if r.index == name:
                        break  # keep arrival order within an index
            keep.extend(self.pending)
            self.pending = keep
            if take:
                self.bytes_in_flight += self._batch_bytes(ix, nq)
            return name, take, nq

    def _launch(self, slot: _Slot, name: str, batch: list, nq: int):
        torch = self.torch
        ix = self.indexes[name]
        W = words(ix.d)
        hq = slot.host_q.view(-1)[:nq * W].view(nq, W)  # contiguous [nq, W] views
        hqn = hq.numpy()
        at = 0
        for r in batch:
            m = r.queries.shape[0]
            hqn[at:at + m] = r.queries.view(np.int64)
            slot.host_r[at:at + m] = r.radius
            at += m
        with torch.cuda.stream(slot.stream):
            q = slot.qbuf.view(-1)[:nq * W].view(nq, W)
            q.copy_(hq, non_blocking=True)
            slot.rbuf[:nq].copy_(slot.host_r[:nq], non_blocking=True)
            ix.query_async(q, ix.info["r"], slot.offsets[:nq + 1], slot.ids, slot.result,
                           radii=slot.rbuf[:nq], stream=slot.stream)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.event, slot.batch, slot.index, slot.nq = ev, batch, name, nq
        slot.keep = q
        self.batches += 1

    def _finish(self, slot: _Slot):
        torch = self.torch
        ix = self.indexes[slot.index]
        res = slot.result.cpu().numpy()
        total, status = int(res[0]), int(res[1])
        if status & (QUERY_IDS_OVERFLOW | QUERY_PAIR_OVERFLOW | QUERY_SPILL_OVERFLOW):
            # rerun this batch synchronously with exact sizing
            with torch.cuda.stream(slot.stream):
                offs, ids = ix.query_radii(slot.keep, slot.rbuf[:slot.nq], stream=slot.stream)
            offs = offs.cpu().numpy()
            ids = ids.cpu().numpy().view(np.uint32)
        else:
            offs = slot.offsets[:slot.nq + 1].cpu().numpy()
            ids = slot.ids[:total].cpu().numpy().view(np.uint32)
        now = time.perf_counter()
        at = 0
        for r in slot.batch:
            m = r.queries.shape[0]
            r.t_done = now
            r.future.set_result([ids[offs[i]:offs[i + 1]].copy() for i in range(at, at + m)])
            self.latencies.append(now - r.t_submit)
            self.completed += 1
            self.queries_done += m
            at += m
        with self.lock:
            self.bytes_in_flight -= self._batch_bytes(ix, slot.nq)
        slot.event = None
        slot.batch = None
        slot.keep = None

    def _loop(self):
        while True:
            idle = True
            for slot in self.slots:
                if slot.event is not None and slot.event.query():
                    self._finish(slot)
                    idle = False
            for slot in self.slots:
                if slot.event is None:
                    name, batch, nq = self._form_batch()
                    if not batch:
                        break
                    self._launch(slot, name, batch, nq)
                    idle = False
            if self.stop_flag and not self.pending and all(s.event is None for s in self.slots):
                return
            if idle:
                time.sleep(20e-6)


def poisson_trace(rate_per_s: float, duration_s: float, rng: np.random.Generator):
    """Arrival times of a Poisson process of the given rate."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            return out
        out.append(t)
