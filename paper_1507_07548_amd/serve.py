"""Continuous-batching request loop over device-resident simulation slots.

Requests (a model family, a system and its MD/sampling settings) arrive over
time.  Each model family owns a backend (a context + batch on its own HIP
stream).  The loop alternates
  1. admission: arrived requests, in arrival order, are admitted while a slot
     is free in their family's batch and the total device footprint of all
     admitted systems stays within the HBM budget (the first request that
     does not fit blocks the ones behind it);
  2. a chunk of `chunk_steps` MD steps for every family with work, launched
     on the families' streams so that their kernels overlap on the device;
  3. completion: slots that reached their step budget (or failed) are
     sampled, retired, and their memory returned to the budget.
Latency of a request = completion time - arrival time (wall clock).

Backends expose footprint / admit / step / sync / poll / collect / retire /
active, so the scheduler runs unchanged against a fake backend on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    model: str              # backend key
    system: Any             # inputs.System (md.n_steps = the request's steps)
    precision: int = 1


@dataclasses.dataclass
class Result:
    rid: int
    model: str
    n: int
    status: int
    steps_done: int
    arrival: float
    admitted: float
    finished: float
    samples: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class GpuBackend:
    """One model family: an ms2 context and batch advanced on its own stream."""

    def __init__(self, species, max_slots: int, stream=None, autotune: Optional[tuple] = None):
        import torch

        from . import ms2
        self.ms2 = ms2
        self.ctx = ms2.Context(species)
        if autotune:
            self.ctx.autotune(*autotune)
        self.batch = ms2.Batch(self.ctx, max_slots)
        self.stream = stream or torch.cuda.Stream()
        self.slots: Dict[int, int] = {}       # slot -> requested steps

    def footprint(self, system, precision) -> int:
        return self.batch.footprint(system, precision)

    def admit(self, system, precision) -> Optional[int]:
        try:
            slot = self.batch.admit(system, precision, stream=self.stream)
        except self.ms2.MS2Error as e:
            if e.status in (2, 5):            # no memory / no slot: try later
                return None
            raise
        self.slots[slot] = system.md.n_steps
        return slot

    def active(self) -> int:
        return len(self.slots)

    def step(self, k: int):
        self.batch.step(k, graph=True, stream=self.stream)

    def sync(self):
        self.stream.synchronize()

    def poll(self):
        out = []
        for slot, target in self.slots.items():
            steps, status = self.batch.status(slot, stream=self.stream)
            out.append((slot, steps, status, steps >= target or status != 0))
        return out

    def collect(self, slot: int) -> dict:
        return self.batch.sample(slot, state=True, stream=self.stream)

    def retire(self, slot: int):
        self.batch.retire(slot)
        self.slots.pop(slot, None)


class Server:
    def __init__(self, backends: Dict[str, Any], hbm_budget: int, chunk_steps: int = 100,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, keep_samples: bool = True):
        self.backends = backends
        self.budget = hbm_budget
        self.chunk = chunk_steps
        self.clock = clock
        self.sleep = sleep
        self.keep_samples = keep_samples
        self.log: List[tuple] = []            # (time, event, rid)

    def run(self, requests: List[Request]) -> List[Result]:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        running: Dict[tuple, tuple] = {}     # (model, slot) -> (request, footprint, admitted)
        used = 0
        results: List[Result] = []
        t0 = self.clock()
        while pending or running:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending[0]
                be = self.backends[r.model]
                fp = be.footprint(r.system, r.precision)
                if used + fp > self.budget:
                    break
                slot = be.admit(r.system, r.precision)
                if slot is None:
                    break
                used += fp
                running[(r.model, slot)] = (r, fp, self.clock() - t0)
                pending.popleft()
                self.log.append((self.clock() - t0, "admit", r.rid))
            if not running:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(wait)
                continue
            busy = [be for be in self.backends.values() if be.active()]
            for be in busy:
                be.step(self.chunk)
            for be in busy:
                be.sync()
            for model, be in self.backends.items():
                if not be.active():
                    continue
                for slot, steps, status, done in be.poll():
                    if not done:
                        continue
                    r, fp, adm = running.pop((model, slot))
                    samples = be.collect(slot) if self.keep_samples else None
                    be.retire(slot)
                    used -= fp
                    t = self.clock() - t0
                    results.append(Result(r.rid, model, r.system.n, status, steps, r.arrival, adm, t, samples))
                    self.log.append((t, "done", r.rid))
        return results


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]
