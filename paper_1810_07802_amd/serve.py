"""Continuous-batching request loop over a serving pool.

Requests (a case to solve for a number of steps) arrive over time. The loop
admits them in arrival order as soon as the pool has a free slot and room in
its arena for the case's state (footprint admission), so requests that arrive
while others run join the running set and their steps overlap on the device
with everybody else's. It advances the pool by fixed chunks of steps, reads
out every case that has reached its step count, and retires it so that its
slot and memory can be reused. It reports each request's time to solution
(arrival to result on the host).

A request whose state turns non-finite (NaN or Inf: the pool reports
ENUMERIC for its slot after a sync) fails alone: it is retired at once with
``error`` set, its slot and memory return to the pool, and every other
request goes on unaffected.

The pool can be the HIP one (``paper_1810_07802_amd.Pool``) or any object
with the same methods (``admit``, ``step``, ``remaining``, ``status``,
``macros``, ``retire``, ``sync``), which is how the scheduling logic is
tested without a GPU.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    case: dict     # nx, ny, params, phi[, u, v, p] (the workloads format)
    steps: int
    arrival: float  # seconds after the start of the run


@dataclass
class Served:
    rid: int
    cells: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    macros: dict | None = field(default=None, repr=False)
    error: str | None = None  # "ENUMERIC": the state went non-finite (no result)

    @property
    def tts(self) -> float:
        """Time to solution: arrival to result on the host."""
        return self.finished - self.arrival


def run(pool, requests, chunk=100, keep=None, use_graph=True, clock=time.perf_counter,
        sleep=time.sleep):
    """Serve ``requests`` on ``pool``; returns the list of ``Served`` in
    completion order. ``keep(request)`` decides whether a result's macros are
    copied back (default: all); ``chunk`` is the number of steps the pool
    advances between two looks at arrivals and completions. With
    ``use_graph`` the pool replays captured HIP graphs, which needs a stream
    set with ``pool.set_stream`` (the null stream cannot be captured)."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    waiting = deque()
    active = {}  # slot -> (request, admission time)
    out = []
    t0 = clock()
    while pending or waiting or active:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # admission in arrival order, by slot and footprint
        while waiting:
            r = waiting[0]
            slot = pool.admit(r.case, r.steps)
            if slot is None:
                if not active:
                    raise RuntimeError(f"request {r.rid} does not fit in an empty pool")
                break
            waiting.popleft()
            active[slot] = (r, now)
        if not active:
            if pending:
                sleep(max(0.0, pending[0].arrival - (clock() - t0)))
            continue
        pool.step(chunk, use_graph)
        # one chunk in flight: the wait keeps the host from queueing ahead of
        # the device, so that new arrivals join at the next chunk; it also
        # brings every slot's numeric status up to date
        pool.sync()
        failed = [s for s in active if pool.status(s) != 0]
        done = [s for s in active if s not in failed and pool.remaining(s) == 0]
        results = {}
        for s in done:
            r, _ = active[s]
            results[s] = pool.macros(s) if (keep is None or keep(r)) else None
        fin = clock() - t0
        for s in failed:
            r, adm = active.pop(s)
            pool.retire(s)
            out.append(Served(r.rid, r.case["nx"] * r.case["ny"], r.steps, r.arrival, adm, fin,
                              None, "ENUMERIC"))
        for s in done:
            r, adm = active.pop(s)
            pool.retire(s)
            out.append(Served(r.rid, r.case["nx"] * r.case["ny"], r.steps, r.arrival, adm, fin,
                              results[s]))
    return out


def summary(served, makespan=None):
    """p50 / p99 time to solution and aggregate MLUPS of a served run."""
    import numpy as np
    ok = [s for s in served if s.error is None]
    tts = np.array([s.tts for s in ok])
    lups = float(sum(s.cells * s.steps for s in ok))
    if makespan is None:
        makespan = max(s.finished for s in served) - min(s.arrival for s in served)
    return {"requests": len(served), "failed": len(served) - len(ok), "p50_s": float(np.percentile(tts, 50)),
            "p99_s": float(np.percentile(tts, 99)), "mlups": lups / makespan / 1e6,
            "makespan_s": makespan}
