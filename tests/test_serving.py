"""Host logic of the continuous-batching scheduler, with a fake executor on a
virtual clock (no GPU): admission by footprint, arrival order, queueing,
cancellation, failure isolation, rejection, latency accounting.  Each test
runs with an executor that only advances whole quanta and checks sims one by
one, and with one that launches a quantum and waits for it separately
(admission overlaps it) and checks sims in one call."""
import dataclasses

import pytest

import workloads
from paper_1301_5892_amd.serving import Scheduler, summarize


class FakeExecutor:
    """Virtual-clock executor: a quantum costs (cells x steps) / rate seconds."""

    def __init__(self, rate=1e9, fail_rids=(), bytes_per_cell=8):
        self.t = 0.0
        self.rate = rate
        self.fail_rids = set(fail_rids)
        self.bpc = bytes_per_cell
        self.live = {}
        self.log = []
        self.max_live_bytes = 0

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def footprint(self, w):
        return w.nx * w.nv * self.bpc

    def start(self, req):
        h = object()
        self.live[h] = [req, 0]
        self.log.append(("start", req.rid, self.t))
        self.max_live_bytes = max(self.max_live_bytes,
                                  sum(self.footprint(r.workload) for r, _ in self.live.values()))
        return h

    def advance(self, handles, counts):
        work = 0
        for h, c in zip(handles, counts):
            req, done = self.live[h]
            assert c > 0 and done + c <= req.workload.nsteps
            self.live[h][1] += c
            work += req.workload.nx * req.workload.nv * c
        self.t += work / self.rate

    def failed(self, h):
        req, done = self.live[h]
        return req.rid in self.fail_rids and done > 0

    def check_quantum(self, handles):
        assert len(set(map(id, handles))) == len(handles)
        assert all(h in self.live for h in handles)

    def finish(self, h):
        req, done = self.live[h]
        assert done == req.workload.nsteps
        return {"rid": req.rid, "steps": done}

    def release(self, h):
        del self.live[h]


class FakeOverlapExecutor(FakeExecutor):
    """Same clock, but launch() only records the quantum and wait() runs it, so
    the scheduler can admit requests in between."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.queued = None
        self.max_stepped = 0

    def start(self, req):
        if self.queued is not None:
            self.log.append(("start_during_quantum", req.rid, self.t))
        return super().start(req)

    def launch(self, handles, counts):
        assert self.queued is None
        self.check_quantum(handles)
        self.queued = (list(handles), list(counts))
        self.max_stepped = max(self.max_stepped, len(handles))

    def wait(self):
        handles, counts = self.queued
        self.queued = None
        FakeExecutor.advance(self, handles, counts)

    def advance(self, handles, counts):
        raise AssertionError("the overlapping executor is driven by launch/wait")

    def failed_many(self, handles):
        assert self.queued is None
        return [self.failed(h) for h in handles]


@pytest.fixture(params=[FakeExecutor, FakeOverlapExecutor], ids=["advance", "overlap"])
def Ex(request):
    return request.param


def mix(n=40, rate=50.0):
    return workloads.serving_mix(n, rate=rate, seed=3, steps_range=(20, 200))


def test_all_requests_complete_in_order_of_admission(Ex):
    reqs = mix()
    ex = Ex()
    out = Scheduler(ex, budget_bytes=1 << 40, max_active=8, quantum=25).run(reqs)
    assert [o.rid for o in out] == sorted(r.rid for r in reqs)
    assert all(o.status == "done" for o in out)
    starts = [rid for kind, rid, _ in ex.log if kind == "start"]
    arrival_order = [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert starts == arrival_order                    # FIFO admission
    for o, r in zip(out, sorted(reqs, key=lambda r: r.rid)):
        assert o.result == {"rid": r.rid, "steps": r.workload.nsteps}
        assert o.admitted >= r.arrival - 1e-12 and o.completed > o.admitted
        assert o.cell_steps == r.workload.nx * r.workload.nv * r.workload.nsteps
    assert not ex.live


def test_budget_is_never_exceeded_and_forces_queueing(Ex):
    reqs = mix()
    ex = Ex()
    budget = max(ex.footprint(r.workload) for r in reqs) * 2
    sched = Scheduler(ex, budget_bytes=budget, max_active=64, quantum=10)
    out = sched.run(reqs)
    assert all(o.status == "done" for o in out)
    assert ex.max_live_bytes <= budget
    assert sched.stats["max_queue"] > 0
    assert sched.stats["max_bytes"] <= budget


def test_slot_limit(Ex):
    reqs = [dataclasses.replace(r, arrival=0.0) for r in mix(20)]
    ex = Ex()
    sched = Scheduler(ex, budget_bytes=1 << 40, max_active=3, quantum=10)
    out = sched.run(reqs)
    assert sched.stats["max_active"] == 3
    assert getattr(ex, "max_stepped", 3) <= 3
    assert all(o.status == "done" for o in out)


def test_overlapped_admission_refills_ending_slots():
    # Two slots, every request one quantum long: while a quantum runs, the two
    # requests after it are admitted into the slots it frees.
    w = workloads.landau_weak().replace(nsteps=10)
    reqs = [workloads.Request(i, 0.0, w) for i in range(6)]
    ex = FakeOverlapExecutor(rate=w.cells * 10.0)      # one request-quantum = 1 s
    out = Scheduler(ex, budget_bytes=1 << 40, max_active=2, quantum=10).run(reqs)
    assert [o.status for o in out] == ["done"] * 6
    during = [rid for kind, rid, _ in ex.log if kind == "start_during_quantum"]
    assert during == [2, 3, 4, 5]
    assert [o.completed for o in out] == pytest.approx([2, 2, 4, 4, 6, 6])
    assert ex.max_stepped == 2


def test_failure_is_isolated(Ex):
    reqs = mix(12)
    ex = Ex(fail_rids={3, 7})
    out = Scheduler(ex, budget_bytes=1 << 40, max_active=4, quantum=10).run(reqs)
    status = {o.rid: o.status for o in out}
    assert status[3] == "failed" and status[7] == "failed"
    assert all(s == "done" for rid, s in status.items() if rid not in (3, 7))
    s = summarize(out)
    assert s["failed"] == 2 and s["done"] == 10


def test_cancellation_frees_the_slot(Ex):
    reqs = [dataclasses.replace(r, arrival=0.0) for r in mix(6)]
    ex = Ex()
    sched = Scheduler(ex, budget_bytes=1 << 40, max_active=1, quantum=5)
    sched.cancel(0)    # running first
    sched.cancel(4)    # still waiting
    out = sched.run(reqs)
    status = {o.rid: o.status for o in out}
    assert status[0] == "cancelled" and status[4] == "cancelled"
    assert sum(s == "done" for s in status.values()) == 4
    assert not ex.live


def test_oversized_request_rejected(Ex):
    reqs = mix(5)
    ex = Ex()
    small = min(ex.footprint(r.workload) for r in reqs)
    out = Scheduler(ex, budget_bytes=small, max_active=4, quantum=10).run(reqs)
    for o, r in zip(out, sorted(reqs, key=lambda r: r.rid)):
        if ex.footprint(r.workload) > small:
            assert o.status == "rejected"
        else:
            assert o.status == "done"


def test_latency_includes_queueing(Ex):
    # Two requests arriving together on one slot: the second waits for the first.
    w = workloads.landau_weak().replace(nsteps=100)
    reqs = [workloads.Request(0, 0.0, w), workloads.Request(1, 0.0, w)]
    ex = Ex(rate=w.cells * 100.0)          # one request = 1 s of work
    out = Scheduler(ex, budget_bytes=1 << 40, max_active=1, quantum=100).run(reqs)
    assert out[0].latency == pytest.approx(1.0)
    assert out[1].latency == pytest.approx(2.0)
    s = summarize(out)
    assert s["p50_latency_s"] == pytest.approx(1.5)
    assert s["aggregate_cell_updates_per_s"] == pytest.approx(w.cells * 100.0)


def test_idle_gap_waits_for_arrival(Ex):
    w = workloads.landau_weak().replace(nsteps=10)
    reqs = [workloads.Request(0, 5.0, w)]
    ex = Ex(rate=w.cells * 10.0)
    out = Scheduler(ex, budget_bytes=1 << 40, max_active=1, quantum=10).run(reqs)
    assert out[0].admitted == pytest.approx(5.0)
    assert out[0].latency == pytest.approx(1.0)


def test_invalid_scheduler_arguments(Ex):
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(), budget_bytes=0)
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(), budget_bytes=1, quantum=0)
