"""Request loop for Stokes solves with continuous batching.

Requests (arrival time, workload) are admitted first-come first-served while
the HBM footprint of their hierarchies (levels, coefficient tables, packed
patch inverses, coarse inverse, Krylov storage; ``stk_footprint``) fits the
budget and a slot is free. An admitted request's hierarchy is built on a
setup thread (its own stream) while the device keeps working on the others;
its solve then joins the running set. Every scheduler tick calls
``stk_step_batch`` on the running solves: a solve whose last phase has
finished on the device gets its host part and its next phase enqueued at
once, without waiting for the others (phases run on the hierarchies' own
streams, so the requests' work overlaps on the device). With
STK_CROSS_BATCH=1 in the environment, the Arnoldi steps of same-shape
requests that are ready together also run in lockstep with one batched
star-patch solve launch per smoothing step of their small levels.
Each request is solved once, so its phases are plain launches: capturing a
HIP graph per Arnoldi step pays off only for repeated solves on one
hierarchy. Finished or failed requests free their memory at once, which
lets waiting requests in; a request that fails (setup, start or solve) is
recorded with its error and the loop goes on. Latency is completion time
minus arrival time (queueing, setup and solve).

The solves run the same kernels in the same order as ``stk_solve`` on each
hierarchy, so a request's result is bit-identical alone and in the mix.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time
from typing import List, Optional, Tuple

from .stk import Hierarchy, StkError, desc_from_workload, stk_footprint, stk_step_batch


def _build_on_own_stream(wl, mixed):
    """Hierarchy of a request, set up on a fresh stream (setup overlaps the
    running solves)."""
    import torch
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = Hierarchy.from_workload(wl, mixed=mixed)
    s.synchronize()
    return h


@dataclasses.dataclass
class Result:
    index: int
    name: str
    unknowns: int
    arrival: float
    admitted: float = 0.0
    started: float = 0.0
    finished: float = 0.0
    iters: int = 0
    converged: bool = False
    rel_res: float = 0.0
    status: int = 0
    footprint: int = 0
    setup_s: float = 0.0
    error: str = ""
    solution: Optional[tuple] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


class Server:
    """Admission by footprint, resident per-request state, per-phase stepping."""

    def __init__(self, hbm_budget: int = 32 << 30, max_active: int = 16, setup_workers: int = 2,
                 mixed: bool = False, keep_solutions: bool = False, rtol: float = 1e-8, eager: bool = True,
                 pc: str = "full", cycle: str = "V", build=None, step=None, footprint=None):
        """build(wl, mixed) -> hierarchy, step(list of hierarchies) and
        footprint(wl, mixed) -> bytes default to the library's own
        (Hierarchy.from_workload on a fresh stream, stk_step_batch,
        stk_footprint); tests pass stand-ins."""
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.setup_workers = int(setup_workers)
        self.mixed = bool(mixed)
        self.keep = bool(keep_solutions)
        self.rtol = rtol
        self.eager = bool(eager)
        self.pc = pc
        self.cycle = cycle
        self._build = build or _build_on_own_stream
        self._step = step or stk_step_batch
        self._footprint = footprint or (lambda wl, mixed: stk_footprint(desc_from_workload(wl, mixed=mixed)))

    def _setup(self, wl):
        t = time.perf_counter()
        h = self._build(wl, 1 if self.mixed else 0)
        return h, time.perf_counter() - t

    def run(self, requests: List[Tuple[float, object]], log=None) -> dict:
        order = sorted(range(len(requests)), key=lambda i: requests[i][0])
        pending = collections.deque(order)
        waiting: collections.deque = collections.deque()
        results = {}
        setups = {}                 # future -> index
        active = []                 # (index, hierarchy, xu, xp)
        used = 0
        peak_used = 0
        peak_active = 0
        ticks = 0
        pool = cf.ThreadPoolExecutor(max_workers=self.setup_workers)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        try:
            while pending or waiting or setups or active:
                t = now()
                while pending and requests[pending[0]][0] <= t:
                    i = pending.popleft()
                    arr, wl = requests[i]
                    n_u, n_p = wl.unknowns()
                    r = Result(i, wl.name, n_u + n_p, arr)
                    r.footprint = self._footprint(wl, 1 if self.mixed else 0)
                    results[i] = r
                    if r.footprint > self.budget:
                        r.error = "footprint exceeds the budget"
                        r.finished = t
                        continue
                    waiting.append(i)
                # admission (first come, first served)
                while waiting and len(active) + len(setups) < self.max_active:
                    i = waiting[0]
                    r = results[i]
                    if used + r.footprint > self.budget:
                        break
                    waiting.popleft()
                    used += r.footprint
                    peak_used = max(peak_used, used)
                    r.admitted = now()
                    setups[pool.submit(self._setup, requests[i][1])] = i
                # finished setups join the running set
                for f in [f for f in setups if f.done()]:
                    i = setups.pop(f)
                    r = results[i]
                    try:
                        h, r.setup_s = f.result()
                    except StkError as e:
                        r.error, r.status, r.finished = str(e), e.status, now()
                        used -= r.footprint
                        continue
                    try:
                        bu, bp = h.stk_rhs()
                        xu, xp = h.stk_solve_begin(bu, bp, rtol=self.rtol, mixed=self.mixed, eager=self.eager,
                                                   pc=self.pc, cycle=self.cycle)
                    except StkError as e:
                        # a request that cannot start (e.g. a non-finite
                        # right-hand side) is recorded and its memory released
                        r.error, r.status, r.finished = str(e), e.status, now()
                        h.close()
                        used -= r.footprint
                        continue
                    r.started = now()
                    active.append((i, h, xu, xp))
                peak_active = max(peak_active, len(active))
                if active:
                    try:
                        self._step([a[1] for a in active])
                    except StkError:
                        pass                    # the failing solve reports through its poll below
                    ticks += 1
                    still = []
                    for i, h, xu, xp in active:
                        r = results[i]
                        try:
                            info = h.stk_poll()
                        except StkError as e:
                            r.error, r.status, r.finished = str(e), e.status, now()
                            h.close()
                            used -= r.footprint
                            if log:
                                log(f"[serve] {r.name}: failed: {e}")
                            continue
                        if info is None:
                            still.append((i, h, xu, xp))
                            continue
                        r.finished = now()
                        r.iters, r.converged, r.rel_res, r.status = (info["iters"], info["converged"],
                                                                      info["rel_res"], info["status"])
                        if self.keep:
                            import torch
                            torch.cuda.synchronize()
                            r.solution = (xu.cpu().numpy(), xp.cpu().numpy())
                        h.close()
                        used -= r.footprint
                        if log:
                            log(f"[serve] {r.name}: {r.iters} it, latency {1e3 * r.latency:.1f} ms")
                    active = still
                else:
                    time.sleep(0.0005)
        finally:
            pool.shutdown(wait=True)
            for _, h, _, _ in active:
                h.close()
        done = [r for r in results.values() if r.converged]
        lat = [r.latency for r in done]
        t_first = min((r.arrival for r in results.values()), default=0.0)
        t_last = max((r.finished for r in results.values()), default=0.0)
        span = max(t_last - t_first, 1e-12)
        return {
            "requests": len(requests), "completed": len(done),
            "failed": len(results) - len(done),
            "dof_per_s": sum(r.unknowns for r in done) / span,
            "makespan_s": span,
            "latency_p50_ms": 1e3 * _percentile(lat, 0.5) if lat else None,
            "latency_p99_ms": 1e3 * _percentile(lat, 0.99) if lat else None,
            "peak_active": peak_active, "peak_footprint_bytes": peak_used, "ticks": ticks,
            "setup_s_mean": sum(r.setup_s for r in done) / max(len(done), 1),
            "solve_s_mean": sum(r.finished - r.started for r in done) / max(len(done), 1),
            "queue_s_mean": sum(r.admitted - r.arrival for r in done) / max(len(done), 1),
            "results": [results[i] for i in sorted(results)],
        }
