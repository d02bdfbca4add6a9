"""Continuous-batching request loop over resident indexes.

Requests (an index name, a block of queries, a radius) arrive at any time.
Up to `streams` batches are in flight on the GPU, one per stream slot.  Each
slot has its own thread: it takes the oldest waiting requests of one index
-- any mix of radii, each query keeping its own -- as one batch of at most
`max_batch` queries, enqueues the library's synchronisation-free batched
path (fclsh_query_batch_async) on its stream, waits for the batch's event,
splits the answers back into the requests (re-running the batch
synchronously on its own stream if a buffer overflowed, which holds up no
other slot) and takes the next batch.  Batches of different slots overlap
on the device; a slot with nothing to do sleeps until a request arrives.
Latency = completion time - submit time.  A request's future resolves to
an Answers object: its queries' neighbour lists as one CSR slice.

Memory admission.  The server holds the indexes resident and reserves, per
slot and index, a query workspace for `max_batch` queries; the bytes each
reservation takes are measured (fclsh_index_memory before and after), and the
server is admitted only if the indexes' own device bytes, every workspace and
the slots' buffers fit `mem_budget` (else ValueError at construction).  A
running server allocates nothing more on the normal path.

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


class Answers:
    """A request's neighbour lists as one CSR slice: answers[i] is the
    uint32 id array of its i-th query (ascending); len() is the number of
    queries."""

    __slots__ = ("offsets", "ids")

    def __init__(self, offsets: np.ndarray, ids: np.ndarray):
        self.offsets = offsets  # int64 [m + 1], from 0
        self.ids = ids          # uint32 [offsets[-1]]

    def __len__(self):
        return len(self.offsets) - 1

    def __getitem__(self, i):
        if not -len(self) <= i < len(self):
            raise IndexError(i)
        i %= len(self)
        return self.ids[self.offsets[i]:self.offsets[i + 1]]

    def __iter__(self):
        return (self[i] for i in range(len(self)))


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
    k: int
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
    keep: object = None


class Server:
    """Serve exact r-NN requests against resident indexes.

    indexes        name -> built Index (kept resident in HBM)
    max_batch      queries per launched batch (also the per-slot capacity)
    streams        batches in flight at once (one HIP stream each)
    mem_budget     device bytes the served set may hold: the indexes, the
                   per-slot query workspaces and the slot buffers
    ids_per_query  result capacity per query of a slot; a batch that does not
                   fit is rerun synchronously with exact sizing
    """

    def __init__(self, indexes: dict, max_batch: int = 4096, streams: int = 3,
                 mem_budget: int = 64 << 30, ids_per_query: int = 64):
        import torch

        self.torch = torch
        self.indexes = dict(indexes)
        self.max_batch = int(max_batch)
        self.mem_budget = int(mem_budget)
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.pending = collections.deque()
        self.stop_flag = False
        self.latencies = []
        self.completed = 0
        self.queries_done = 0
        self.batches = 0
        self.reruns = 0
        # the indexes' own device bytes (points, tables, directory, kept
        # build scratch, workspaces they already hold)
        self.index_bytes = {}
        for name, ix in self.indexes.items():
            m = ix.memory()
            self.index_bytes[name] = m["index_bytes"] + m["build_scratch_bytes"] + m["workspace_bytes"]
        wmax = max(words(ix.d) for ix in self.indexes.values())
        cap = self.max_batch * ids_per_query
        slot_bytes = (self.max_batch * wmax * 8 + self.max_batch * 4 + (self.max_batch + 1) * 8 + cap * 4 + 16)
        self.workspace_bytes = {}
        self.resident_bytes = sum(self.index_bytes.values()) + streams * slot_bytes
        if self.resident_bytes > self.mem_budget:
            raise ValueError(f"indexes need {self.resident_bytes} bytes, over the budget of {self.mem_budget}")
        self.slots = []
        for k in range(streams):
            st = torch.cuda.Stream()
            slot = _Slot(
                k=k, stream=st,
                qbuf=torch.empty((self.max_batch, wmax), dtype=torch.int64, device="cuda"),
                rbuf=torch.empty(self.max_batch, dtype=torch.int32, device="cuda"),
                offsets=torch.empty(self.max_batch + 1, dtype=torch.int64, device="cuda"),
                ids=torch.empty(cap, dtype=torch.int32, device="cuda"),
                result=torch.zeros(2, dtype=torch.int64, device="cuda"),
                host_q=torch.empty((self.max_batch, wmax), dtype=torch.int64, pin_memory=True),
                host_r=torch.empty(self.max_batch, dtype=torch.int32, pin_memory=True),
            )
            for name, ix in self.indexes.items():
                before = ix.memory()["workspace_bytes"]
                ix.reserve(self.max_batch, pair_capacity=cap, spill_capacity=1 << 18, stream=st)
                grown = ix.memory()["workspace_bytes"] - before
                self.workspace_bytes[(k, name)] = grown
                self.resident_bytes += grown
                if self.resident_bytes > self.mem_budget:
                    raise ValueError(f"query workspaces take the served set to {self.resident_bytes} bytes, "
                                     f"over the budget of {self.mem_budget}")
            self.slots.append(slot)
        self.threads = [threading.Thread(target=self._serve_slot, args=(s,), daemon=True) for s in self.slots]
        for t in self.threads:
            t.start()

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
        with self.cv:
            self.pending.append(req)
            self.cv.notify_all()
        return req.future

    def close(self):
        """Stop once every submitted request is answered."""
        with self.cv:
            self.stop_flag = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    def stats(self) -> dict:
        with self.lock:
            lat = np.asarray(self.latencies, np.float64)
            return {"requests": self.completed, "queries": self.queries_done, "batches": self.batches,
                    "reruns": self.reruns, "resident_bytes": self.resident_bytes,
                    "p50_ms": float(np.percentile(lat, 50)) * 1e3 if lat.size else None,
                    "p99_ms": float(np.percentile(lat, 99)) * 1e3 if lat.size else None,
                    "mean_ms": float(lat.mean()) * 1e3 if lat.size else None}

    # ------------------------------------------------------------ internals
    def _form_batch(self):
        """Oldest waiting requests of the oldest request's index, within
        max_batch queries, keeping arrival order within an index.  Called
        with the lock held."""
        if not self.pending:
            return None, [], 0
        name = self.pending[0].index
        take, nq, keep = [], 0, collections.deque()
        while self.pending:
            r = self.pending.popleft()
            m = r.queries.shape[0]
            if r.index == name and nq + m <= self.max_batch:
                take.append(r)
                nq += m
            else:
                keep.append(r)
                if r.index == name:
                    break
        keep.extend(self.pending)
        self.pending = keep
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
        slot.event, slot.batch, slot.index, slot.nq, slot.keep = ev, batch, name, nq, q

    def _finish(self, slot: _Slot):
        """Answers of the slot's finished batch to its requests."""
        torch = self.torch
        slot.event.synchronize()
        ix = self.indexes[slot.index]
        res = slot.result.cpu().numpy()
        total, status = int(res[0]), int(res[1])
        rerun = bool(status & (QUERY_IDS_OVERFLOW | QUERY_PAIR_OVERFLOW | QUERY_SPILL_OVERFLOW))
        if rerun:
            # rerun this batch synchronously with exact sizing, on this
            # slot's stream (the other slots keep running)
            with torch.cuda.stream(slot.stream):
                offs, ids = ix.query_radii(slot.keep, slot.rbuf[:slot.nq], stream=slot.stream)
            offs = offs.cpu().numpy()
            ids = ids.cpu().numpy().view(np.uint32)
        else:
            offs = slot.offsets[:slot.nq + 1].cpu().numpy()
            ids = slot.ids[:total].cpu().numpy().view(np.uint32)
        now = time.perf_counter()
        at = 0
        lats = []
        for r in slot.batch:
            m = r.queries.shape[0]
            r.t_done = now
            o = offs[at:at + m + 1]
            r.future.set_result(Answers(o - o[0], ids[o[0]:o[-1]].copy()))
            lats.append(now - r.t_submit)
            at += m
        with self.lock:
            self.latencies.extend(lats)
            self.completed += len(slot.batch)
            self.queries_done += slot.nq
            self.reruns += int(rerun)
        slot.event = slot.batch = slot.keep = None

    def _serve_slot(self, slot: _Slot):
        while True:
            with self.cv:
                while not self.pending and not self.stop_flag:
                    self.cv.wait()
                if not self.pending:
                    return  # stopped, nothing left
                name, batch, nq = self._form_batch()
                self.batches += 1
            self._launch(slot, name, batch, nq)
            self._finish(slot)


def poisson_trace(rate_per_s: float, duration_s: float, rng: np.random.Generator):
    """Arrival times of a Poisson process of the given rate."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            return out
        out.append(t)
