"""Continuous-batching request loop over device-resident simulation slots.

Requests (a model family, a system and its MD/sampling settings) arrive over
time.  Each model family owns a backend (a context + batch on its own HIP
stream), and every family progresses on its own: the loop repeatedly
  1. completion: for each family whose last chunk of MD steps has finished
     on the device, slots that reached their step budget (or failed) are
     sampled, retired, and their memory returned to the budget;
  2. admission: arrived requests, in arrival order, are admitted into their
     family's batch while it is idle (no chunk in flight), a slot is free
     and the total device footprint of all admitted systems stays within the
     HBM budget.  The first request that does not fit the budget blocks the
     ones behind it; a family that is busy or full holds back its own later
     requests only.  A request that can never run -- larger than the whole
     budget, or refused by its backend while nothing at all is running -- is
     returned at once as a failed result with the backend's status;
  3. launch: idle families with active slots start their next chunk of
     `chunk_steps` steps on their own streams.  Without a limit every idle
     family launches, so the families' kernels overlap on the device.  With
     `max_inflight` = k, at most k families have a chunk on the device, and
     the idle ones launch in order of estimated remaining work, shortest
     first: the remaining steps of the family's nearest request times the
     family's cost per step, the sum of `cost(request)` (default n^2, the
     pair count) over its running requests.  Shortest-remaining-work order
     minimises the mean completion time of a set of jobs; it matters here
     because the kernels of a batch of large systems fill every compute
     unit, so a batch of small systems on another stream gains little from
     running beside them and would otherwise finish at the large ones'
     pace.  The order is revised at every chunk boundary, the only place a
     family can be held back.
Latency of a request = completion time - arrival time (wall clock).

Backends expose footprint / admit / active / launch / ready / poll / collect
/ retire, so the scheduler runs unchanged against a fake backend on the CPU.
"""
from __future__ import annotations

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
        self.event = torch.cuda.Event()
        self.slots: Dict[int, int] = {}       # slot -> requested steps
        self.last_status = 0

    def footprint(self, system, precision) -> int:
        return self.batch.footprint(system, precision)

    def admit(self, system, precision) -> Optional[int]:
        try:
            slot = self.batch.admit(system, precision, stream=self.stream)
        except self.ms2.MS2Error as e:
            if e.status in (2, 5):            # no memory / no slot: try later
                self.last_status = e.status
                return None
            raise
        self.slots[slot] = system.md.n_steps
        return slot

    def active(self) -> int:
        return len(self.slots)

    def launch(self, k: int):
        """Enqueue k steps of every active slot (asynchronous)."""
        self.batch.step(k, graph=True, stream=self.stream)
        self.event.record(self.stream)

    def ready(self) -> bool:
        """True once the last launched chunk has finished on the device."""
        return self.event.query()

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
                 sleep: Callable[[float], None] = time.sleep, keep_samples: bool = True,
                 poll_s: float = 2e-4, max_inflight: Optional[int] = None,
                 cost: Callable[[Request], float] = lambda r: float(r.system.n) ** 2):
        if max_inflight is not None and max_inflight < 1:
            raise ValueError("max_inflight must be >= 1 (or None for no limit)")
        self.backends = backends
        self.max_inflight = max_inflight
        self.cost = cost
        self.budget = hbm_budget
        self.chunk = chunk_steps
        self.clock = clock
        self.sleep = sleep
        self.keep_samples = keep_samples
        self.poll_s = poll_s
        self.log: List[tuple] = []            # (time, event, rid)

    def run(self, requests: List[Request]) -> List[Result]:
        pending: List[Request] = sorted(requests, key=lambda r: (r.arrival, r.rid))
        running: Dict[tuple, list] = {}      # (model, slot) -> [request, footprint, admitted, steps launched]
        inflight = set()                      # families with a chunk on the device
        used = 0
        results: List[Result] = []
        t0 = self.clock()

        def finish(r, status, steps, admitted, samples=None):
            t = self.clock() - t0
            results.append(Result(r.rid, r.model, r.system.n, status, steps, r.arrival, admitted, t, samples))
            self.log.append((t, "done" if status == 0 else "failed", r.rid))

        while pending or running:
            progressed = False
            # 1. completions of families whose chunk has finished
            for model, be in self.backends.items():
                if model not in inflight or not be.ready():
                    continue
                inflight.discard(model)
                progressed = True
                for slot, steps, status, done in be.poll():
                    if not done:
                        continue
                    r, fp, adm, _ = running.pop((model, slot))
                    samples = be.collect(slot) if self.keep_samples else None
                    be.retire(slot)
                    used -= fp
                    finish(r, status, steps, adm, samples)
            # 2. admission in arrival order
            now = self.clock() - t0
            held = set()                      # families that keep their later requests back
            keep: List[Request] = []
            stop = False
            for idx, r in enumerate(pending):
                if stop or r.arrival > now:
                    keep.extend(pending[idx:])
                    break
                if r.model in held:
                    keep.append(r)
                    continue
                be = self.backends[r.model]
                fp = be.footprint(r.system, r.precision)
                if fp > self.budget:          # can never fit: fail it now
                    finish(r, 2, 0, now)
                    progressed = True
                    continue
                if used + fp > self.budget:   # the budget blocks everything behind it
                    keep.extend(pending[idx:])
                    break
                if r.model in inflight:
                    held.add(r.model)
                    keep.append(r)
                    continue
                slot = be.admit(r.system, r.precision)
                if slot is None:
                    if not running and not inflight:   # nothing will ever free room for it
                        finish(r, getattr(be, "last_status", 5) or 5, 0, now)
                        progressed = True
                        continue
                    held.add(r.model)
                    keep.append(r)
                    continue
                used += fp
                running[(r.model, slot)] = [r, fp, self.clock() - t0, 0]
                self.log.append((self.clock() - t0, "admit", r.rid))
                progressed = True
            pending = keep
            # 3. idle families with work start their next chunk
            idle = [m for m, be in self.backends.items() if m not in inflight and be.active()]
            if self.max_inflight is not None:
                idle.sort(key=lambda m: self._remaining_work(m, running))
                idle = idle[:max(0, self.max_inflight - len(inflight))]
            for model in idle:
                self.backends[model].launch(self.chunk)
                inflight.add(model)
                for key, entry in running.items():
                    if key[0] == model:
                        entry[3] += self.chunk
                progressed = True
            if not running and pending:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(wait)
                continue
            if not progressed:
                self.sleep(self.poll_s)
        return results

    def _remaining_work(self, model: str, running: Dict[tuple, list]) -> float:
        """Estimated work until the family's nearest request completes: its
        remaining steps (requested - launched) times the family's cost per
        step.  Slots of a batch step in lockstep, so every running request of
        the family pays that cost for every step."""
        entries = [e for key, e in running.items() if key[0] == model]
        if not entries:
            return float("inf")
        per_step = sum(self.cost(e[0]) for e in entries)
        nearest = min(max(1, e[0].system.md.n_steps - e[3]) for e in entries)
        return nearest * per_step


# bounds of the size classes, in molecules: class k holds
# SIZE_CLASSES[k-1] <= n < SIZE_CLASSES[k]
# (a bound at 2048 keeps the lighter medium systems out of the batch of the
# 2048-4095 ones: in the configured trace the median request then finishes
# with that batch at 8-9.5 s instead of at 15-20 s)
SIZE_CLASSES = (1024, 2048, 4096)


def size_class(n: int, classes=SIZE_CLASSES) -> int:
    return sum(1 for b in classes if n >= b)


def backend_key(model: str, n: int, classes=SIZE_CLASSES) -> str:
    """The batch a request of `model` with n molecules joins: one per model
    family and size class.  The slots of a batch step in lockstep, so a small
    request sharing a batch with a large one would finish at the large one's
    pace; with a batch per size class it runs at its own."""
    return f"{model}/{size_class(n, classes)}"


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]
