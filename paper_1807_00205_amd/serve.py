"""Continuous-batching search server over a resident index.

Requests (query spans) arrive at any time.  Each request reserves device
memory for its search; a request is admitted when its reservation fits the
HBM budget next to the reservations of the requests already on the GPU.
Worker threads, each owning one HIP stream, take every queued request that
fits and run them as one batched search, so requests that arrive while
others are on the GPU join the next batch and batches of different workers
overlap on the device.  The library holds each batched search to the sum of
its requests' reservations (``sdf_search_batch_capped``): a search never
takes more device memory than was admitted.  A batch that would need more
fails without allocating it; its requests go back to the head of the queue
with four times their reservation.  Every request's result is the candidate
set of its span alone (query ids are local to the request).

Reservations start from an estimate per query base and are kept at least
1.25 times the most any finished search needed per base: the device memory
of a search grows with its seeds, which cannot be bounded usefully in
advance (a hit can start a seed in every window that holds its minimizer,
so the count of hits times the windows per minimizer overshoots the real
need by one to three orders of magnitude).

The plain mode (``workers=1, max_batch=1``) is the one-request-at-a-time
FIFO baseline.  ``tuning`` (settings for ``sdf.set_tuning``, such as the
schedule ``Index.autotune`` returns) is installed in every worker thread.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import sdf

MIN_RESERVE = 8 << 20       # bytes reserved for any request
START_BYTES_PER_BASE = 40.0  # first estimate, raised by what searches report


def request_bytes(span_len: int, per_base: float = START_BYTES_PER_BASE) -> int:
    """Device memory reserved for one request of span_len query bases."""
    return max(MIN_RESERVE, int(span_len * per_base))


_STREAMS: dict = {}


def worker_streams(n: int):
    """n HIP streams (default priority) kept for the life of the process, so
    that the device memory the library caches per stream is found again by
    every later server instead of being allocated anew."""
    import torch
    dev = torch.cuda.current_device()
    lst = _STREAMS.setdefault(dev, [])
    while len(lst) < n:
        lst.append(torch.cuda.Stream())
    return lst[:n]


class Request:
    __slots__ = ("span", "arrival", "future", "bytes")

    def __init__(self, span, arrival, nbytes):
        self.span = span
        self.arrival = arrival
        self.future = Future()
        self.bytes = nbytes


class Server:
    def __init__(self, index: sdf.Index, workers: int = 2, max_batch: int = 4096,
                 hbm_budget: Optional[int] = None, max_error: float = 0.25,
                 min_len: int = 1000, tuning: Optional[dict] = None):
        import torch
        self.index = index
        self.tuning = dict(tuning or {})
        self.max_batch = max_batch
        self.max_error, self.min_len = max_error, min_len
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.5)
        self.budget = hbm_budget
        self.per_base = START_BYTES_PER_BASE
        self.in_flight = 0
        self.queue: collections.deque = collections.deque()
        self.cv = threading.Condition()
        self.stop = False
        self.batches = []   # (size, seconds) per batch
        self.retries = 0    # batches that needed more than their reservation
        self.streams = worker_streams(workers)
        self.threads = [threading.Thread(target=self._work, args=(s,), daemon=True)
                        for s in self.streams]
        for t in self.threads:
            t.start()

    def submit(self, span: Tuple[int, int, int], arrival: Optional[float] = None) -> Future:
        with self.cv:
            nbytes = request_bytes(span[2] - span[1], self.per_base)
        r = Request(span, time.perf_counter() if arrival is None else arrival, nbytes)
        if r.bytes > self.budget:
            r.future.set_exception(MemoryError("request exceeds the HBM budget"))
            return r.future
        with self.cv:
            self.queue.append(r)
            self.cv.notify()
        return r.future

    def _take(self) -> List[Request]:
        """Admit queued requests in arrival order while the budget allows."""
        batch = []
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            if self.in_flight + r.bytes > self.budget:
                break
            self.queue.popleft()
            self.in_flight += r.bytes
            batch.append(r)
        return batch

    def _work(self, stream):
        sdf.set_tuning(**self.tuning)  # the settings are per thread
        while True:
            with self.cv:
                while not self.stop and not (self.queue and
                                             self.in_flight + self.queue[0].bytes <= self.budget):
                    self.cv.wait()
                if self.stop and not self.queue:
                    return
                batch = self._take()
            if not batch:
                continue
            t0 = time.perf_counter()
            reserved = sum(r.bytes for r in batch)
            retry = []
            peak = 0
            try:
                res, peak = self.index.search_batch_capped(
                    [r.span for r in batch], reserved, self.max_error, self.min_len,
                    stream=stream)
                c = res.candidates()
                res.close()
                done = time.perf_counter()
                order = np.argsort(c["query_id"], kind="stable")
                c = c[order]
                bounds = np.searchsorted(c["query_id"], np.arange(len(batch) + 1))
                for q, r in enumerate(batch):
                    mine = c[bounds[q]:bounds[q + 1]].copy()
                    mine["query_id"] = 0
                    r.future.set_result((mine, done))
            except sdf.SdfError as e:
                done = time.perf_counter()
                if e.code == sdf.SDF_ENOMEM:
                    retry = batch  # nothing was kept: admitted again with more room
                else:
                    for r in batch:
                        r.future.set_exception(e)
            except Exception as e:  # isolate failures per batch
                done = time.perf_counter()
                for r in batch:
                    if not r.future.done():
                        r.future.set_exception(e)
            with self.cv:
                self.in_flight -= reserved
                self.batches.append((len(batch), done - t0))
                bases = sum(r.span[2] - r.span[1] for r in batch)
                if peak and not retry and bases:
                    self.per_base = max(self.per_base, 1.25 * peak / bases)
                if retry:
                    self.retries += 1
                    for r in reversed(retry):
                        r.bytes *= 4
                        if r.bytes > self.budget:
                            r.future.set_exception(MemoryError("request exceeds the HBM budget"))
                        else:
                            self.queue.appendleft(r)
                self.cv.notify_all()

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()


def open_loop(server: Server, requests: Sequence[Tuple[float, Tuple[int, int, int]]]):
    """Submit (arrival offset in s, span) pairs at their arrival times and
    wait for all; returns per-request latencies (s), query bases and the
    wall time from the first arrival to the last completion."""
    t0 = time.perf_counter()
    futs = []
    for (ta, span) in requests:
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        arr = time.perf_counter()
        futs.append((arr, span, server.submit(span, arr)))
    lat, bases, last = [], 0, t0
    for arr, span, f in futs:
        _, done = f.result()
        lat.append(done - arr)
        bases += span[2] - span[1]
        last = max(last, done)
    first = futs[0][0] if futs else t0
    return np.array(lat), bases, last - first


def measure(index: sdf.Index, requests, workers: int, max_batch: int, **kw):
    srv = Server(index, workers=workers, max_batch=max_batch, **kw)
    try:
        lat, bases, wall = open_loop(srv, requests)
    finally:
        srv.close()
    sizes = [b for b, _ in srv.batches]
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mbp_per_s": bases / wall / 1e6 if wall > 0 else 0.0,
            "requests": len(lat), "batches": len(sizes),
            "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "retries": srv.retries, "bytes_per_base": round(srv.per_base, 2)}
