"""Continuous-batching request loop for many Vlasov-Poisson simulations.

Requests (a workload each) arrive over time.  The scheduler keeps every
admitted simulation's f and E resident in device memory, admits waiting
requests in arrival order whenever a slot is free and the summed device
footprint (vog_workspace_bytes of each sim) stays within the budget, and
advances all active simulations together in quanta of Strang steps with
grouped launches (vog_step_batch: one launch per kernel type and line length
across the whole active set).  Finished, failed or cancelled simulations are
retired between quanta, which frees their memory and slot for the next
admission.  Latency of a request = completion time - arrival time.

With an executor that can launch a quantum and wait for it separately
(`launch`, `wait`), admission also runs while a quantum executes: the slots of
simulations that complete in that quantum are refilled then (their memory is
still counted against the budget), and the new simulations join the next
quantum, so creating them overlaps the device work.

The scheduler talks to an executor; `GpuExecutor` drives libvog on the
current torch stream.  Per-simulation arithmetic does not depend on which
other simulations share a launch, so each result equals the result of the
same request run alone.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import time
from collections import deque
from typing import Any, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Outcome:
    rid: int
    status: str                 # "done", "failed", "cancelled", "rejected"
    arrival: float
    admitted: Optional[float]
    completed: Optional[float]
    cell_steps: int
    result: Any = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.completed is None else self.completed - self.arrival


@dataclasses.dataclass
class _Active:
    req: Any
    handle: Any
    remaining: int
    footprint: int
    admitted: float


class Scheduler:
    """Admission by memory footprint + quantum-based continuous batching."""

    def __init__(self, executor, budget_bytes: int, max_active: int = 64, quantum: int = 50,
                 check_every: int = 4):
        if budget_bytes <= 0 or max_active <= 0 or quantum <= 0 or check_every <= 0:
            raise ValueError("budget, max_active, quantum and check_every must be positive")
        # a simulation's field is checked for non-finite values every
        # check_every quanta and when it completes (each check synchronises)
        self.check_every = int(check_every)
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.quantum = int(quantum)
        self.cancelled: set = set()
        self.stats = {"quanta": 0, "max_active": 0, "max_bytes": 0, "max_queue": 0}

    def cancel(self, rid: int) -> None:
        self.cancelled.add(rid)

    def run(self, requests: Sequence[Any]) -> List[Outcome]:
        """Serve `requests` (each with .rid, .arrival, .workload), arrival
        times in seconds relative to the start of the run."""
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: deque = deque()
        active: List[_Active] = []
        outcomes: Dict[int, Outcome] = {}
        used = 0
        t0 = self.ex.now()
        overlap = hasattr(self.ex, "launch") and hasattr(self.ex, "wait")

        def now() -> float:
            return self.ex.now() - t0

        def intake() -> None:
            nonlocal waiting
            tnow = now()
            while pending and pending[0].arrival <= tnow:
                waiting.append(pending.popleft())
            # cancellations of waiting requests
            if self.cancelled:
                keep = deque()
                for r in waiting:
                    if r.rid in self.cancelled:
                        outcomes[r.rid] = Outcome(r.rid, "cancelled", r.arrival, None, tnow, 0)
                    else:
                        keep.append(r)
                waiting = keep

        def admit(into: List[_Active], slots: int) -> None:
            # admission in arrival order into at most `slots` free slots
            nonlocal used
            while waiting and slots > 0:
                r = waiting[0]
                fp = self.ex.footprint(r.workload)
                if fp > self.budget:
                    waiting.popleft()
                    outcomes[r.rid] = Outcome(r.rid, "rejected", r.arrival, None, now(), 0)
                    continue
                if used + fp > self.budget:
                    break
                waiting.popleft()
                h = self.ex.start(r)
                into.append(_Active(r, h, r.workload.nsteps, fp, now()))
                used += fp
                slots -= 1
            self.stats["max_bytes"] = max(self.stats["max_bytes"], used)

        incoming: List[_Active] = []
        while pending or waiting or active or incoming:
            active.extend(incoming)
            incoming = []
            intake()
            admit(active, self.max_active - len(active))
            self.stats["max_active"] = max(self.stats["max_active"], len(active))
            self.stats["max_queue"] = max(self.stats["max_queue"], len(waiting))
            if not active:
                if pending:
                    self.ex.wait_until(t0 + pending[0].arrival)
                continue
            # one quantum for every active sim
            counts = [min(self.quantum, a.remaining) for a in active]
            if overlap:
                self.ex.launch([a.handle for a in active], counts)
                ending = sum(c == a.remaining for a, c in zip(active, counts))
                intake()
                admit(incoming, self.max_active - (len(active) - ending))
                self.ex.wait()
            else:
                self.ex.advance([a.handle for a in active], counts)
            self.stats["quanta"] += 1
            check = self.stats["quanta"] % self.check_every == 0
            tq = now()
            for a, c in zip(active, counts):
                a.remaining -= c
            # non-finite checks: every check_every quanta and at completion,
            # one call for all of them when the executor offers it
            probe = [a for a in active if a.req.rid not in self.cancelled
                     and (a.remaining == 0 or check)]
            bad = set()
            if probe:
                if hasattr(self.ex, "failed_many"):
                    flags = self.ex.failed_many([a.handle for a in probe])
                else:
                    flags = [self.ex.failed(a.handle) for a in probe]
                bad = {id(a) for a, f in zip(probe, flags) if f}
            still: List[_Active] = []
            for a in active:
                rid = a.req.rid
                w = a.req.workload
                if rid in self.cancelled:
                    status = "cancelled"
                elif id(a) in bad:
                    status = "failed"
                elif a.remaining == 0:
                    status = "done"
                else:
                    still.append(a)
                    continue
                res = self.ex.finish(a.handle) if status == "done" else None
                done_steps = w.nsteps - a.remaining
                outcomes[rid] = Outcome(rid, status, a.req.arrival, a.admitted, tq,
                                        w.nx * w.nv * done_steps, res)
                self.ex.release(a.handle)
                used -= a.footprint
            active = still
        return [outcomes[k] for k in sorted(outcomes)]


class GpuExecutor:
    """Runs requests with libvog on the current torch stream."""

    def __init__(self, moments_every: int = 0, keep_state: bool = False, digest: bool = False):
        import torch

        from . import vog
        self.torch = torch
        self.vog = vog
        self.moments_every = moments_every
        self.keep_state = keep_state
        self.digest = digest
        vog.load()

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float) -> None:
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    def footprint(self, w) -> int:
        return self.vog.workspace_bytes(self.vog.make_config(w, self.moments_every))

    def start(self, req):
        return self.vog.Sim(req.workload, moments_every=self.moments_every).init()

    def launch(self, handles, counts) -> None:
        """Enqueues one quantum (grouped by step count) without waiting."""
        groups: Dict[int, list] = {}
        for h, c in zip(handles, counts):
            groups.setdefault(c, []).append(h)
        for c, hs in sorted(groups.items(), reverse=True):
            self.vog.step_batch(hs, c)

    def wait(self) -> None:
        self.torch.cuda.synchronize()

    def advance(self, handles, counts) -> None:
        self.launch(handles, counts)
        self.wait()

    def failed(self, h) -> bool:
        try:
            h.sync()
            return False
        except self.vog.VogError as e:
            if e.code == self.vog.ENONFINITE:
                return True
            raise

    def failed_many(self, handles) -> List[bool]:
        return [not ok for ok in self.vog.sync_batch(handles)]

    def finish(self, h):
        """Result of a finished request: the final field and step count; the
        stored f (keep_state) and its SHA-256 (digest) on request."""
        out = {"E": h.get_E(), "step": h.time()[0]}
        if self.keep_state or self.digest:
            raw = h.get_raw()
            if self.digest:
                out["digest"] = hashlib.sha256(raw.tobytes()).hexdigest()
            if self.keep_state:
                out["raw"] = raw
        return out

    def release(self, h) -> None:
        h.close()
        h.workspace = None


def summarize(outcomes: Sequence[Outcome]) -> Dict[str, Any]:
    done = [o for o in outcomes if o.status == "done"]
    lat = np.array([o.latency for o in done]) if done else np.zeros(0)
    work = sum(o.cell_steps for o in outcomes)
    if done:
        first = min(o.arrival for o in outcomes)
        last = max(o.completed for o in outcomes if o.completed is not None)
        span = last - first
    else:
        span = float("nan")
    return {
        "requests": len(outcomes),
        "done": len(done),
        "failed": sum(o.status == "failed" for o in outcomes),
        "cancelled": sum(o.status == "cancelled" for o in outcomes),
        "rejected": sum(o.status == "rejected" for o in outcomes),
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_latency_s": float(lat.mean()) if lat.size else None,
        "cell_updates": int(work),
        "makespan_s": span,
        "aggregate_cell_updates_per_s": work / span if span and span > 0 else None,
    }


def bench(n_requests: int = 512, load_factors: Sequence[float] = (0.5, 0.8, 1.0, 1.2),
          headline_load: float = 0.8, quantum: int = 25, max_active: int = 128,
          budget_bytes: int = 64 << 30, binding_fraction: float = 0.25,
          seed: int = 1) -> Dict[str, Any]:
    """Serving mix: a closed-loop capacity pass (all requests present at t=0),
    open-loop passes with Poisson arrivals at each of load_factors x capacity
    (p50/p99 latency at each; the headline fields are those at headline_load),
    and one more pass at headline_load with a budget of binding_fraction of
    the peak bytes that pass held, so that admission by memory footprint
    binds and requests queue."""
    import workloads

    ex = GpuExecutor()
    # warm the kernels of every line length used by the mix
    warm = workloads.serving_mix(min(n_requests, 32), rate=1e9, seed=seed,
                                 steps_range=(2, 2))
    Scheduler(ex, budget_bytes, max_active, quantum).run(warm)

    reqs0 = workloads.serving_mix(n_requests, rate=1.0, seed=seed)
    closed = [dataclasses.replace(r, arrival=0.0) for r in reqs0]
    t0 = time.perf_counter()
    res_closed = Scheduler(ex, budget_bytes, max_active, quantum).run(closed)
    cap_time = time.perf_counter() - t0
    capacity = n_requests / cap_time              # requests per second
    s_closed = summarize(res_closed)

    def open_pass(load: float, budget: int) -> Dict[str, Any]:
        reqs = workloads.serving_mix(n_requests, rate=load * capacity, seed=seed)
        sched = Scheduler(ex, budget, max_active, quantum)
        s = summarize(sched.run(reqs))
        return {"load_factor": load, "arrival_rate_per_s": load * capacity,
                "p50_latency_s": s["p50_latency_s"], "p99_latency_s": s["p99_latency_s"],
                "mean_latency_s": s["mean_latency_s"],
                "aggregate_cell_updates_per_s": s["aggregate_cell_updates_per_s"],
                "done": s["done"], "failed": s["failed"], "budget_bytes": budget,
                "max_active": sched.stats["max_active"], "max_queue": sched.stats["max_queue"],
                "max_bytes": sched.stats["max_bytes"]}

    sweep = [open_pass(lf, budget_bytes) for lf in load_factors]
    head = next((p for p in sweep if p["load_factor"] == headline_load), None)
    if head is None:
        head = open_pass(headline_load, budget_bytes)
    largest = max(ex.footprint(r.workload) for r in reqs0)
    binding = open_pass(headline_load, max(largest, int(binding_fraction * head["max_bytes"])))
    return {
        "requests": n_requests,
        "arrival_rate_per_s": head["arrival_rate_per_s"],
        "load_factor": headline_load,
        "closed_loop_capacity_req_per_s": capacity,
        "closed_loop_aggregate_cell_updates_per_s": s_closed["aggregate_cell_updates_per_s"],
        "p50_latency_s": head["p50_latency_s"],
        "p99_latency_s": head["p99_latency_s"],
        "mean_latency_s": head["mean_latency_s"],
        "aggregate_cell_updates_per_s": head["aggregate_cell_updates_per_s"],
        "done": head["done"],
        "failed": head["failed"],
        "quantum_steps": quantum,
        "max_active": head["max_active"],
        "max_queue": head["max_queue"],
        "budget_bytes": budget_bytes,
        "load_sweep": sweep,
        "binding_budget": binding,
    }
