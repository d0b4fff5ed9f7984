"""Request server for Crank-Nicolson solves with continuous batching.

Requests (an AMR hierarchy, B and eta per level, dt) arrive over time.  The
server keeps *slots* resident in HBM: a slot is a single-problem handle for
one request shape (base box, cell width, block lists), device buffers for B
and eta of that shape, and the step's workspace.  A request is admitted when
an idle slot of its shape exists, or when the HBM budget left over by every
resident slot (busy or idle) fits a new one, after evicting idle slots of
other shapes, least recently used first.  Admission is first come, first
served.

``n_streams`` workers, each with its own HIP stream, take admitted requests
one at a time: the request's fields go into its slot through pinned host
memory (asynchronous copies on the worker's stream), the step runs, the result
comes back the same way.  The step synchronises its stream once per outer
iteration, so the outer iterations of all requests in flight interleave on
the device: a request that arrives while others are being solved starts as
soon as a worker is free, and its iterations run between theirs.  A slot keeps
its workspace and field pointers, so the step's captured graphs are replayed
for every request of that shape and repeated shapes build no handle.  Each
result equals the same request solved alone (same single-problem handle,
every reduction per problem in a fixed order); a request's ``result`` arrays
are views of pinned host buffers of its own.

All arithmetic runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import ctypes
import dataclasses
import threading
import time
from collections import OrderedDict, deque

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
    slot_reused: bool = False

    @property
    def cells(self) -> int:
        tot = 0
        for l, blk in enumerate(self.levels):
            n = len(blk) * 512
            if l + 1 < len(self.levels):
                n -= len(self.levels[l + 1]) * 64
            tot += n
        return tot


def shape_key(req: Request):
    """Requests with equal keys share slots: same base box, cell width and
    block lists."""
    blk = b"".join(np.ascontiguousarray(l, dtype=np.int32).tobytes() + b"|" for l in req.levels)
    return (tuple(int(b) for b in req.base_blocks), float(req.dx0), blk)


def _workspace_bytes(h: Hierarchy, opts) -> int:
    nb = ctypes.c_size_t()
    _lib.check(_lib.lib().ohm_cn_workspace_size(h.h, ctypes.byref(opts), ctypes.byref(nb)))
    return int(nb.value)


def _field_bytes(req: Request) -> int:
    return sum(4 * len(blk) * 512 * 8 for blk in req.levels)


def footprint(req: Request, opts) -> int:
    """Device bytes of a slot for the request's shape: the handle's own
    memory, B and eta, and the step's workspace (a throwaway handle sizes it)."""
    import torch
    h = Hierarchy([(req.base_blocks, req.dx0, req.levels)], torch.cuda.current_stream())
    try:
        return h.device_bytes() + _field_bytes(req) + _workspace_bytes(h, opts) + 256
    finally:
        h.close()


class Slot:
    """A resident single-problem handle with B, eta and workspace on the device
    and pinned host staging for the inputs."""

    def __init__(self, req: Request, opts, stream):
        import torch
        self.key = shape_key(req)
        self.h = Hierarchy([(req.base_blocks, req.dx0, req.levels)], stream)
        nb = [len(l) for l in req.levels]
        self.B = [torch.empty((3, n, 8, 8, 8), dtype=torch.float64, device="cuda") for n in nb]
        self.E = [torch.empty((1, n, 8, 8, 8), dtype=torch.float64, device="cuda") for n in nb]
        self.pin_B = [torch.empty((3, n, 8, 8, 8), dtype=torch.float64, pin_memory=True) for n in nb]
        self.pin_E = [torch.empty((1, n, 8, 8, 8), dtype=torch.float64, pin_memory=True) for n in nb]
        self.ws = Workspace()
        self.ws.get(_workspace_bytes(self.h, opts))
        self.bytes = self.h.device_bytes() + _field_bytes(req) + self.ws.buf.numel()
        self.last_used = 0.0

    def solve(self, req: Request, opts, stream):
        """The request's step in this slot on `stream`; returns (status,
        stats, results as views of new pinned buffers)."""
        import torch
        with torch.cuda.stream(stream):
            for l in range(len(self.B)):
                self.pin_B[l].copy_(torch.from_numpy(np.ascontiguousarray(req.B[l])))
                self.pin_E[l][0].copy_(torch.from_numpy(np.ascontiguousarray(req.eta[l])))
                self.B[l].copy_(self.pin_B[l], non_blocking=True)
                self.E[l].copy_(self.pin_E[l], non_blocking=True)
            st, stats = ohm_cn_step(self.h, self.B, self.E, req.dt, opts, self.ws, stream=stream)
            out = []
            for b in self.B:
                o = torch.empty(b.shape, dtype=b.dtype, pin_memory=True)
                o.copy_(b, non_blocking=True)
                out.append(o)
            stream.synchronize()
        return st, stats, [o.numpy() for o in out]

    def close(self):
        self.h.close()
        self.B = self.E = self.pin_B = self.pin_E = None
        self.ws.buf = None


class Server:
    def __init__(self, hbm_budget: int, n_streams: int = 4, precision: int = 1, rtol: float = 1e-10, **schedule):
        """``schedule``: further ``ohm_cn_opts`` fields (nu_pre, nu_post,
        nu_coarse, cycle, outer, ...) applied to every request."""
        self.budget = int(hbm_budget)
        self.resident = 0                   # bytes of resident slots (busy, idle or being built)
        self.n_streams = n_streams
        self.opts = default_opts(rtol=rtol, precision=precision, max_iters=300, **schedule)
        self.lock = threading.Condition()
        self.waiting: deque = deque()       # arrived, not admitted
        self.admitted: deque = deque()      # admitted, not started
        self.assigned: dict = {}            # rid -> idle slot it will reuse (None: a new slot)
        self.idle: OrderedDict = OrderedDict()   # (key, id) -> idle slot, least recently used first
        self.to_close: list = []            # evicted slots, closed by a worker
        self.finished: list = []
        self.closed = False
        self.streams = None                 # one HIP stream per worker, made by serve()
        self.t0 = time.perf_counter()
        self.fp: dict = {}                  # shape key -> slot bytes
        self.keys: dict = {}                # rid -> shape key
        self.built = 0                      # slots built
        self.reused = 0                     # requests served by an idle slot

    @property
    def free(self) -> int:
        return self.budget - self.resident

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- admission -------------------------------------------------------------
    def submit(self, req: Request):
        # sizing builds a throwaway handle for a shape seen the first time:
        # done outside the lock so that workers are not held up; a request the
        # library rejects (blocks outside the base grid, improper nesting ...)
        # finishes with its status
        key = shape_key(req)
        fp, err = self.fp.get(key), None
        if fp is None:
            try:
                fp = footprint(req, self.opts)
            except _lib.OhmError as e:
                err = e
        with self.lock:
            if err is None and fp > self.budget:
                err = _lib.OhmError(_lib.OHM_ERR_NOMEM, f"footprint {fp} B exceeds the budget {self.budget} B")
            if err is not None:
                req.status, req.error = err.status, str(err)
                req.done = self.now()
                self.finished.append(req)
                return
            self.fp[key] = fp
            self.keys[req.rid] = key
            self.waiting.append(req)
            self._admit()
            self.lock.notify_all()

    def _idle_of(self, key):
        for k in self.idle:
            if k[0] == key:
                return k
        return None

    def _admit(self):
        """First come, first served: the head request takes an idle slot of
        its shape, or room for a new one (idle slots of other shapes are
        evicted, least recently used first)."""
        while self.waiting:
            r = self.waiting[0]
            key = self.keys[r.rid]
            k = self._idle_of(key)
            if k is not None:
                slot = self.idle.pop(k)
                self.assigned[r.rid] = slot
            else:
                need = self.fp[key]
                while self.free < need and self.idle:
                    _, old = self.idle.popitem(last=False)
                    self.resident -= old.bytes
                    self.to_close.append(old)
                if self.free < need:
                    return
                self.resident += need
                self.assigned[r.rid] = None
            self.waiting.popleft()
            r.admitted = self.now()
            self.admitted.append(r)

    def cancel(self, rid: int) -> bool:
        """Drop a request that has not started; a slot it had is released."""
        with self.lock:
            for q in (self.waiting, self.admitted):
                for r in list(q):
                    if r.rid == rid:
                        q.remove(r)
                        if q is self.admitted:
                            self._release(r, self.assigned.pop(rid))
                        r.status = -2
                        r.done = self.now()
                        self.finished.append(r)
                        self._admit()
                        self.lock.notify_all()
                        return True
        return False

    def _release(self, r, slot):
        """Back into the idle pool (a slot), or the reservation returned."""
        if slot is None:
            self.resident -= self.fp[self.keys[r.rid]]
        else:
            slot.last_used = self.now()
            self.idle[(slot.key, id(slot))] = slot

    # -- workers ---------------------------------------------------------------
    def _take(self):
        with self.lock:
            while not self.admitted and not (self.closed and not self.waiting):
                self.lock.wait(timeout=0.05)
            if not self.admitted:
                return None, None, []
            r = self.admitted.popleft()
            slot = self.assigned.pop(r.rid)
            if slot is None:
                # a slot of its shape may have become idle since admission:
                # take it and return the reservation
                k = self._idle_of(self.keys[r.rid])
                if k is not None:
                    slot = self.idle.pop(k)
                    self.resident -= self.fp[self.keys[r.rid]]
            closing, self.to_close = self.to_close, []
            return r, slot, closing

    def _make_slot(self, req, stream):
        return Slot(req, self.opts, stream)

    def _solve(self, req, slot, stream):
        return slot.solve(req, self.opts, stream)

    def _worker(self, k):
        stream = self.streams[k]
        while True:
            r, slot, closing = self._take()
            for s in closing:
                s.close()
            if r is None:
                return
            r.started = self.now()
            reused = slot is not None
            built = False
            try:
                if slot is None:
                    slot = self._make_slot(r, stream)
                    built = True
                    with self.lock:
                        # the reservation becomes the slot's own size
                        self.resident += slot.bytes - self.fp[self.keys[r.rid]]
                        self.built += 1
                st, stats, out = self._solve(r, slot, stream)
                r.result, r.stats = out, stats[0]
                r.status = 0 if stats[0]["rel_res"] <= self.opts.rtol else _lib.OHM_ERR_NOCONV
                r.slot_reused = reused
            except Exception as e:
                # a request that raises finishes with the error; its slot (if
                # built) is closed and its memory returned, the worker goes on
                r.status = getattr(e, "status", _lib.OHM_ERR_HIP)
                r.error, r.result, r.stats = str(e), None, None
                if slot is not None:
                    slot.close()
                    with self.lock:
                        self.resident -= slot.bytes
                    slot = None
                else:
                    with self.lock:
                        self.resident -= self.fp[self.keys[r.rid]]
            r.done = self.now()
            with self.lock:
                if reused:
                    self.reused += 1
                if slot is not None:
                    slot.last_used = r.done
                    self.idle[(slot.key, id(slot))] = slot
                self.finished.append(r)
                self._admit()
                self.lock.notify_all()

    def serve(self, requests, arrival_times):
        """Feed ``requests`` at ``arrival_times`` (seconds from now) and serve
        them; returns the finished requests.  Idle slots stay resident for a
        later call."""
        import torch
        if self.streams is None:
            self.streams = [torch.cuda.Stream() for _ in range(self.n_streams)]
        self.t0 = time.perf_counter()
        self.closed = False
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

    def shutdown(self):
        """Close every idle slot and return its memory."""
        with self.lock:
            slots = list(self.idle.values())
            self.idle.clear()
            for s in slots:
                self.resident -= s.bytes
            slots += self.to_close
            self.to_close = []
        for s in slots:
            s.close()


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def latency_report(finished) -> dict:
    ok = [r for r in finished if r.status == 0]
    lat = np.array([r.done - r.arrival for r in ok]) if ok else np.zeros(1)
    span = (max(r.done for r in ok) - min(r.arrival for r in ok)) if ok else 1.0
    return {"completed": len(ok), "rejected": sum(1 for r in finished if r.status not in (0,)),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "cells_per_s": float(sum(r.cells for r in ok) / max(span, 1e-9)),
            "requests_per_s": float(len(ok) / max(span, 1e-9))}
