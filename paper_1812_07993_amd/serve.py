"""Continuous-batching server for pore-MD simulation requests.

Requests (a system and a number of steps) arrive over time.  The server keeps
one batch per precision resident on the device, each on its own HIP stream
so their work overlaps, creates systems for arrived requests (on worker
threads if asked: upload and first force evaluation off the tick path),
admits them by device footprint as slots and memory free up, keeps every
busy batch a chunk or two ahead, and reads finished systems back as soon as
a completed chunk shows them done, without waiting for queued work.

Latency of a request = time its results were read back - its arrival time.
All simulation work runs in the library's kernels; this module only
schedules (the Server class documents the loop).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    index: int
    arrival: float          # seconds after the start of the trace
    precision: str          # "mixed" or "fp64"
    steps: int
    n: int                  # vapour atoms (for accounting)
    payload: Any = None     # whatever the backend needs to create the system


@dataclass
class Result:
    index: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    n: int
    precision: str
    status: str = "ok"
    output: Dict[str, Any] = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class PoremdBackend:
    """The library through its C interface (one batch per precision, each on
    its own HIP stream).  Systems are created on library-owned streams, so a
    worker thread can create one while the batches run."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 256, tuning=None,
                 keep_positions: bool = False):
        import torch

        from . import poremd

        self.torch = torch
        self.pm = poremd
        self.pm.load()
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.tuning = tuning
        self.keep_positions = keep_positions
        self._streams = {p: torch.cuda.Stream() for p in ("mixed", "fp64")}
        self._events: Dict[int, deque] = {}

    def new_batch(self, precision: str):
        b = self.pm.pmd_batch_create(self.budget, self.max_slots,
                                     self._streams[precision].cuda_stream)
        self._events[id(b)] = (self._streams[precision], deque())
        return b

    def footprint(self, req: Request) -> int:
        params, pore = self.pm.params_of(req.payload, req.precision)
        return self.pm.pmd_footprint_bytes(params, pore, req.n, self.tuning)

    def create(self, req: Request):
        return self.pm.System.from_desc(req.payload, precision=req.precision,
                                        tuning=self.tuning)

    def admit(self, batch, handle, steps: int) -> Optional[int]:
        return self.pm.pmd_batch_admit(batch, handle.h, steps)

    def advance(self, batch, chunk: int) -> None:
        self.pm.pmd_batch_advance(batch, chunk)
        stream, evs = self._events[id(batch)]
        ev = self.torch.cuda.Event()
        ev.record(stream)
        evs.append(ev)

    def queued(self, batch) -> int:
        """Chunks of this batch the device has not finished yet."""
        _, evs = self._events[id(batch)]
        while evs and evs[0].query():
            evs.popleft()
        return len(evs)

    def poll(self, batch, wait: bool = True) -> List[int]:
        return self.pm.pmd_batch_poll(batch) if wait else self.pm.pmd_batch_poll_async(batch)

    def release(self, batch, slot: int, handle):
        self.pm.pmd_batch_release(batch, slot)
        return handle

    def finish(self, handle) -> Dict[str, Any]:
        out = {"energies": handle.energies()}
        if self.keep_positions:
            out["positions"] = handle.positions()
            out["velocities"] = handle.velocities()
        return out

    def destroy(self, handle) -> None:
        handle.close()

    def destroy_batch(self, batch) -> None:
        self._events.pop(id(batch), None)
        self.pm.pmd_batch_destroy(batch)


class Server:
    """Continuous batching.  Every tick it

      1. starts creating arrived requests, oldest first, whose device
         footprint fits the precision's budget beside the systems already
         resident, ready or being created (a request that does not fit
         waits; later ones that fit may pass it); with create_workers > 0
         the creation (upload and first force evaluation) runs on worker
         threads, off the tick path;
      2. admits created systems into their precision's batch;
      3. keeps up to max_queued chunks of chunk_steps steps queued on each
         batch that holds systems, so the device never waits for the host;
      4. polls each batch without waiting (the systems that had finished by
         the end of the newest completed chunk), reads the finished systems
         back and frees their slots.
    """

    def __init__(self, backend, chunk_steps: int = 250,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 create_workers: int = 0, max_queued: int = 2, idle_sleep: float = 0.0005):
        self.backend = backend
        self.chunk = chunk_steps
        self.clock = clock
        self.sleep = sleep
        self.workers = create_workers
        self.max_queued = max_queued
        self.idle_sleep = idle_sleep
        self.batches: Dict[str, Any] = {}
        self.log: List[str] = []

    def _batch(self, precision):
        if precision not in self.batches:
            self.batches[precision] = self.backend.new_batch(precision)
        return self.batches[precision]

    def run(self, requests: List[Request]) -> List[Result]:
        from concurrent.futures import ThreadPoolExecutor

        be = self.backend
        pool = ThreadPoolExecutor(max_workers=self.workers) if self.workers > 0 else None
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        arrived: List[Request] = []
        creating: List[tuple] = []          # (req, future)
        ready: deque = deque()              # (req, handle or exception)
        resident: Dict[tuple, tuple] = {}   # (precision, slot) -> (req, handle, admitted)
        held = {}                           # precision -> [bytes, systems] not yet released
        results: List[Result] = []
        budget = getattr(be, "budget", 0)
        fp_cache: Dict[int, int] = {}

        def fp(req):
            if req.index not in fp_cache:
                fp_cache[req.index] = be.footprint(req)
            return fp_cache[req.index]

        t0 = self.clock()
        try:
            while pending or arrived or creating or ready or resident:
                now = self.clock() - t0
                while pending and pending[0].arrival <= now:
                    arrived.append(pending.popleft())
                progress = False
                # 1. creations, oldest first, within the budget and the slots
                still = []
                for req in arrived:
                    used, count = held.get(req.precision, (0, 0))
                    f = fp(req)
                    if count >= be.max_slots or (budget and used + f > budget):
                        if count == 0 and budget and f > budget:
                            raise RuntimeError("request %d cannot fit an empty batch" % req.index)
                        still.append(req)
                        continue
                    held[req.precision] = (used + f, count + 1)
                    if pool is not None:
                        creating.append((req, pool.submit(be.create, req)))
                    else:
                        try:
                            ready.append((req, be.create(req)))
                        except Exception as e:  # a failing request must not stop the others
                            ready.append((req, e))
                    progress = True
                arrived = still
                # 2. finished creations, then admission in arrival order
                keep = []
                for req, fut in creating:
                    if fut.done():
                        try:
                            ready.append((req, fut.result()))
                        except Exception as e:
                            ready.append((req, e))
                        progress = True
                    else:
                        keep.append((req, fut))
                creating = keep
                unadmitted = deque()
                while ready:
                    req, h = ready.popleft()
                    if isinstance(h, Exception):
                        t = self.clock() - t0
                        results.append(Result(req.index, req.arrival, t, t, req.steps, req.n,
                                              req.precision, "error", {"error": str(h)}))
                        used, count = held[req.precision]
                        held[req.precision] = (used - fp(req), count - 1)
                        continue
                    slot = be.admit(self._batch(req.precision), h, req.steps)
                    if slot is None:
                        unadmitted.append((req, h))
                        continue
                    resident[(req.precision, slot)] = (req, h, self.clock() - t0)
                    progress = True
                ready = unadmitted
                if not resident:
                    if not (creating or ready):
                        if pending:
                            self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                            continue
                        if arrived:
                            raise RuntimeError("request %d cannot be admitted" % arrived[0].index)
                        break
                    if not progress:
                        self.sleep(self.idle_sleep)
                    continue
                # 3. keep the batches busy
                active = sorted({p for (p, _) in resident})
                for p in active:
                    b = self.batches[p]
                    if be.queued(b) < self.max_queued:
                        be.advance(b, self.chunk)
                        progress = True
                # 4. finished systems (no wait)
                for p in active:
                    for slot in be.poll(self.batches[p], wait=False):
                        if (p, slot) not in resident:
                            continue
                        req, h, t_adm = resident.pop((p, slot))
                        be.release(self.batches[p], slot, h)
                        try:
                            out = be.finish(h)
                            status = "ok"
                        except Exception as e:  # a failing request must not stop the others
                            out, status = {"error": str(e)}, "error"
                        t_fin = self.clock() - t0
                        results.append(Result(req.index, req.arrival, t_adm, t_fin, req.steps,
                                              req.n, p, status, out))
                        be.destroy(h)
                        used, count = held[p]
                        held[p] = (used - fp(req), count - 1)
                        progress = True
                if not progress:
                    self.sleep(self.idle_sleep)
        finally:
            if pool is not None:
                pool.shutdown(wait=True)
            for b in self.batches.values():
                be.destroy_batch(b)
            self.batches = {}
        return sorted(results, key=lambda r: r.index)


def summarize(results: List[Result]) -> Dict[str, float]:
    lat = np.array([r.latency for r in results])
    work = float(sum(r.n * r.steps for r in results))
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "makespan_s": span, "atom_steps": work,
            "atom_steps_per_s": work / span if span > 0 else 0.0,
            "errors": sum(r.status != "ok" for r in results)}


class FakeBackend:
    """CPU stand-in with a virtual clock: a step of a system of n atoms costs
    n * cost_per_atom_step seconds; systems in one batch run concurrently
    (a chunk costs the time of the largest resident system).  For testing
    the scheduling logic without a GPU."""

    def __init__(self, budget: int, max_slots: int, cost_per_atom_step=1e-9,
                 bytes_per_atom=1000, fail_indices=()):
        self.budget = budget
        self.max_slots = max_slots
        self.cost = cost_per_atom_step
        self.bpa = bytes_per_atom
        self.t = 0.0
        self.fail = set(fail_indices)
        self.peak_used = 0

    # clock interface for Server
    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += dt

    def new_batch(self, precision):
        return {"slots": {}, "precision": precision}

    def footprint(self, req):
        return req.n * self.bpa

    def create(self, req):
        return {"req": req, "done": 0}

    def admit(self, b, h, steps):
        used = sum(x["req"].n * self.bpa for x in b["slots"].values())
        if len(b["slots"]) >= self.max_slots or used + h["req"].n * self.bpa > self.budget:
            return None
        slot = next(s for s in range(self.max_slots) if s not in b["slots"])
        b["slots"][slot] = h
        self.peak_used = max(self.peak_used, used + h["req"].n * self.bpa)
        return slot

    def advance(self, b, chunk):
        live = [h for h in b["slots"].values() if h["done"] < h["req"].steps]
        if not live:
            return
        self.t += max(min(chunk, h["req"].steps - h["done"]) * h["req"].n for h in live) * self.cost
        for h in live:
            h["done"] = min(h["req"].steps, h["done"] + chunk)

    def queued(self, b):
        return 0  # a chunk completes in virtual time when it is advanced

    def poll(self, b, wait=True):
        return [s for s, h in b["slots"].items() if h["done"] >= h["req"].steps]

    def release(self, b, slot, h):
        del b["slots"][slot]
        return h

    def finish(self, h):
        if h["req"].index in self.fail:
            raise RuntimeError("non-finite state")
        return {"steps": h["done"]}

    def destroy(self, h):
        pass

    def destroy_batch(self, b):
        pass
