"""Request server for Crank-Nicolson solves with continuous batching.

Requests (an AMR hierarchy, B and eta per level, dt) arrive over time.  A
request is admitted once its device footprint (fields plus solver workspace)
fits in the HBM budget that completed requests have released.  Each of
``n_streams`` workers takes every admitted request that is waiting when it
becomes free, builds one multi-problem handle for them, and runs the step on
its own HIP stream; a batch that arrives while another is on the GPU starts
on the next free stream, so their work overlaps on the device.  Results stay
bitwise equal to a solve alone: every reduction is per problem in a fixed
order.  Fields travel through pinned host buffers in both directions; a
request's ``result`` arrays are views of its batch's pinned output buffer,
which stays allocated until every result of the batch has been released.

All arithmetic runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import ctypes
import dataclasses
import threading
import time
from collections import deque

import numpy as np

from . import _lib
from . import Hierarchy, Workspace, default_opts, ohm_cn_step


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds on the server clock
    base_blocks: tuple
    dx0: float
    levels: list                   # int32 [nb, 3] per level
    B: list                        # numpy [3, nb, 8, 8, 8] per level
    eta: list                      # numpy [nb, 8, 8, 8] per level
    dt: float
    # filled by the server
    admitted: float = -1.0
    started: float = -1.0
    done: float = -1.0
    result: list | None = None
    stats: dict | None = None
    status: int = -1
    error: str = ""

    @property
    def cells(self) -> int:
        tot = 0
        for l, blk in enumerate(self.levels):
            n = len(blk) * 512
            if l + 1 < len(self.levels):
                n -= len(self.levels[l + 1]) * 64
            tot += n
        return tot


def footprint(req: Request, opts) -> int:
    """Device bytes of one request solved alone: B and eta per level plus the
    solver workspace."""
    import torch
    h = Hierarchy([(req.base_blocks, req.dx0, req.levels)], torch.cuda.current_stream())
    nb = ctypes.c_size_t()
    _lib.check(_lib.lib().ohm_cn_workspace_size(h.h, ctypes.byref(opts), ctypes.byref(nb)))
    h.close()
    fields = sum(4 * len(blk) * 512 * 8 for blk in req.levels)
    return int(nb.value) + fields


class Server:
    def __init__(self, hbm_budget: int, n_streams: int = 2, max_batch: int = 32, precision: int = 1,
                 rtol: float = 1e-10, **schedule):
        """``schedule``: further ``ohm_cn_opts`` fields (nu_pre, nu_post,
        nu_coarse, cycle, outer) applied to every batch."""
        self.budget = int(hbm_budget)
        self.free = int(hbm_budget)
        self.n_streams = n_streams
        self.max_batch = max_batch
        self.opts = default_opts(rtol=rtol, precision=precision, max_iters=300, **schedule)
        self.lock = threading.Condition()
        self.waiting: deque = deque()       # arrived, not admitted
        self.admitted: deque = deque()      # admitted, not started
        self.finished: list = []
        self.closed = False
        self.streams = None             # one HIP stream per worker, made by serve()
        self.t0 = time.perf_counter()
        self.fp: dict = {}

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- admission -------------------------------------------------------------
    def submit(self, req: Request):
        # sizing builds a throwaway handle: done outside the lock so that
        # workers are not held up; a request the library rejects (blocks
        # outside the base grid, improper nesting ...) finishes with its status
        try:
            fp, err = footprint(req, self.opts), None
        except _lib.OhmError as e:
            fp, err = None, e
        with self.lock:
            if err is None and fp > self.budget:
                err = _lib.OhmError(_lib.OHM_ERR_NOMEM, f"footprint {fp} B exceeds the budget {self.budget} B")
            if err is not None:
                req.status, req.error = err.status, str(err)
                req.done = self.now()
                self.finished.append(req)
                return
            self.fp[req.rid] = fp
            self.waiting.append(req)
            self._admit()
            self.lock.notify_all()

    def _admit(self):
        while self.waiting and self.fp[self.waiting[0].rid] <= self.free:
            r = self.waiting.popleft()
            self.free -= self.fp[r.rid]
            r.admitted = self.now()
            self.admitted.append(r)

    def cancel(self, rid: int) -> bool:
        """Drop a request that has not started; its budget is released."""
        with self.lock:
            for q in (self.waiting, self.admitted):
                for r in list(q):
                    if r.rid == rid:
                        q.remove(r)
                        if q is self.admitted:
                            self.free += self.fp[rid]
                        r.status = -2
                        r.done = self.now()
                        self.finished.append(r)
                        self._admit()
                        self.lock.notify_all()
                        return True
        return False

    # -- workers ---------------------------------------------------------------
    def _take_batch(self):
        with self.lock:
            while not self.admitted and not (self.closed and not self.waiting):
                self.lock.wait(timeout=0.05)
            if not self.admitted:
                return None
            batch = []
            while self.admitted and len(batch) < self.max_batch:
                batch.append(self.admitted.popleft())
            return batch

    def _run_batch(self, batch, stream, ws):
        import torch
        t_start = self.now()
        for r in batch:
            r.started = t_start
        with torch.cuda.stream(stream):
            h = Hierarchy([(r.base_blocks, r.dx0, r.levels) for r in batch], stream)
            try:
                # the requests' fields are gathered into pinned host buffers and
                # copied asynchronously on this worker's stream (pageable copies
                # run at a fraction of the link's rate); results come back the
                # same way and are handed out as views of the pinned buffers
                nlev = max(len(r.levels) for r in batch)
                B, E = [], []
                for l in range(nlev):
                    bl = [r.B[l] for r in batch if l < len(r.levels)]
                    el = [r.eta[l] for r in batch if l < len(r.levels)]
                    hb = torch.empty((3, sum(b.shape[1] for b in bl)) + bl[0].shape[2:], dtype=torch.float64,
                                     pin_memory=True)
                    torch.cat([torch.from_numpy(b) for b in bl], dim=1, out=hb)
                    he = torch.empty((sum(e.shape[0] for e in el),) + el[0].shape[1:], dtype=torch.float64,
                                     pin_memory=True)
                    torch.cat([torch.from_numpy(e) for e in el], dim=0, out=he)
                    he = he[None]
                    B.append(hb.to("cuda", non_blocking=True))
                    E.append(he.to("cuda", non_blocking=True))
                st, stats = ohm_cn_step(h, B, E, [r.dt for r in batch], self.opts, ws, stream=stream)
                pinned_out = []
                for b in B:
                    o = torch.empty(b.shape, dtype=b.dtype, pin_memory=True)
                    o.copy_(b, non_blocking=True)
                    pinned_out.append(o)
                stream.synchronize()
                outs = [o.numpy() for o in pinned_out]
            finally:
                h.close()           # hipFree inside waits for the device
        off = [0] * nlev
        done = self.now()
        for i, r in enumerate(batch):
            r.result = []
            for l in range(len(r.levels)):
                nb = len(r.levels[l])
                r.result.append(outs[l][:, off[l]:off[l] + nb])
                off[l] += nb
            r.stats = stats[i]
            r.status = 0 if stats[i]["rel_res"] <= self.opts.rtol else _lib.OHM_ERR_NOCONV
            r.done = done

    def _finish(self, batch):
        """Return the batch's budget, record its requests, admit what now fits."""
        with self.lock:
            for r in batch:
                self.free += self.fp[r.rid]
                self.finished.append(r)
            self._admit()
            self.lock.notify_all()

    def _worker(self, k):
        ws = Workspace()
        while True:
            batch = self._take_batch()
            if batch is None:
                return
            try:
                self._run_batch(batch, self.streams[k], ws)
            except Exception as e:
                # a batch that raises ends each of its requests with the error;
                # the worker and the batch's budget stay in service
                now = self.now()
                for r in batch:
                    r.status = getattr(e, "status", _lib.OHM_ERR_HIP)
                    r.error, r.result, r.stats, r.done = str(e), None, None, now
            self._finish(batch)
            ws.buf = None       # release the workspace between batches

    def serve(self, requests, arrival_times):
        """Feed ``requests`` at ``arrival_times`` (seconds from now) and serve
        them; returns the finished requests."""
        import torch
        if self.streams is None:
            self.streams = [torch.cuda.Stream() for _ in range(self.n_streams)]
        self.t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(k,), daemon=True) for k in range(self.n_streams)]
        for w in workers:
            w.start()
        for r, t in zip(requests, arrival_times):
            delay = t - self.now()
            if delay > 0:
                time.sleep(delay)
            r.arrival = self.now()
            self.submit(r)
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        for w in workers:
            w.join()
        return sorted(self.finished, key=lambda r: r.rid)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def latency_report(finished) -> dict:
    ok = [r for r in finished if r.status == 0]
    lat = np.array([r.done - r.arrival for r in ok]) if ok else np.zeros(1)
    span = (max(r.done for r in ok) - min(r.arrival for r in ok)) if ok else 1.0
    return {"completed": len(ok), "rejected": sum(1 for r in finished if r.status not in (0,)),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "cells_per_s": float(sum(r.cells for r in ok) / max(span, 1e-9))}
