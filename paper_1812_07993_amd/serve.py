"""Continuous-batching server for pore-MD simulation requests.

Requests (a system and a number of steps) arrive over time.  The server keeps
one batch per precision resident on the device, each on its own HIP stream
so their work overlaps; every tick it

  1. admits arrived requests, oldest first, as slots and device memory free
     up (admission by footprint: the batch's budget bounds its bytes; a
     request that does not fit waits, later ones that fit may pass it);
  2. advances every batch by a chunk of steps (asynchronous);
  3. polls for finished systems, reads them back and frees their slots.

Latency of a request = time its results were read back - its arrival time.
All simulation work runs in the library's kernels; this module only
schedules.
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
    """The library through its C interface (one batch per precision)."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 256, tuning=None,
                 keep_positions: bool = False):
        import torch

        from . import poremd

        self.pm = poremd
        self.pm.load()
        self.budget = hbm_budget
        self.max_slots = max_slots
        self.tuning = tuning
        self.keep_positions = keep_positions
        self._streams = {p: torch.cuda.Stream() for p in ("mixed", "fp64")}

    def new_batch(self, precision: str):
        return self.pm.pmd_batch_create(self.budget, self.max_slots,
                                        self._streams[precision].cuda_stream)

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

    def poll(self, batch) -> List[int]:
        return self.pm.pmd_batch_poll(batch)

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
        self.pm.pmd_batch_destroy(batch)


class Server:
    def __init__(self, backend, chunk_steps: int = 250,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.backend = backend
        self.chunk = chunk_steps
        self.clock = clock
        self.sleep = sleep
        self.batches: Dict[str, Any] = {}
        self.log: List[str] = []

    def _batch(self, precision):
        if precision not in self.batches:
            self.batches[precision] = self.backend.new_batch(precision)
        return self.batches[precision]

    def run(self, requests: List[Request]) -> List[Result]:
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: List[Request] = []
        resident: Dict[tuple, tuple] = {}   # (precision, slot) -> (req, handle, admitted)
        results: List[Result] = []
        t0 = self.clock()
        while pending or waiting or resident:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # 1. admission, oldest first; a cheap footprint check first so no
            #    system is created on the device only to be turned away
            still = []
            for req in waiting:
                b = self._batch(req.precision)
                fp = self.backend.footprint(req)
                used = sum(self.backend.footprint(r) for (p, _), (r, _, _) in resident.items()
                           if p == req.precision)
                count = sum(1 for (p, _) in resident if p == req.precision)
                budget = getattr(self.backend, "budget", 0)
                if count >= self.backend.max_slots or (budget and used + fp > budget):
                    still.append(req)
                    continue
                h = self.backend.create(req)
                slot = self.backend.admit(b, h, req.steps)
                if slot is None:
                    self.backend.destroy(h)
                    still.append(req)
                    continue
                resident[(req.precision, slot)] = (req, h, self.clock() - t0)
            waiting = still
            if not resident:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                    continue
                if waiting:
                    raise RuntimeError("request %d cannot fit an empty batch" % waiting[0].index)
                break
            # 2. advance every batch holding systems (their streams overlap)
            active = sorted({p for (p, _) in resident})
            for p in active:
                self.backend.advance(self.batches[p], self.chunk)
            # 3. collect finished systems
            for p in active:
                for slot in self.backend.poll(self.batches[p]):
                    req, h, t_adm = resident.pop((p, slot))
                    self.backend.release(self.batches[p], slot, h)
                    try:
                        out = self.backend.finish(h)
                        status = "ok"
                    except Exception as e:  # a failing request must not stop the others
                        out, status = {"error": str(e)}, "error"
                    t_fin = self.clock() - t0
                    results.append(Result(req.index, req.arrival, t_adm, t_fin, req.steps,
                                          req.n, p, status, out))
                    self.backend.destroy(h)
        for b in self.batches.values():
            self.backend.destroy_batch(b)
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

    def poll(self, b):
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
