"""GPU serving: each request's result is the same alone and in the mix, a
diverged request fails without touching the others, and the latency summary
is filled."""
import dataclasses

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def small_mix(n=12):
    # the serving mix's full range of grid sizes: nx 64 .. 1024, nv 128 .. 2048
    reqs = workloads.serving_mix(n, rate=1e6, seed=7, steps_range=(20, 60),
                                 nx_pow=(6, 10), nv_pow=(7, 11))
    return reqs


def test_alone_equals_mix_bitwise(gpu):
    from paper_1301_5892_amd import serving, vog
    reqs = small_mix()
    ex = serving.GpuExecutor(keep_state=True)
    budget = 3 * max(ex.footprint(r.workload) for r in reqs)      # forces queueing
    sched = serving.Scheduler(ex, budget_bytes=budget, max_active=6, quantum=7)
    out = sched.run(reqs)
    assert all(o.status == "done" for o in out)
    assert sched.stats["max_queue"] > 0 and sched.stats["max_active"] >= 2
    sizes = {(r.workload.nx, r.workload.nv) for r in reqs}
    assert max(nx for nx, _ in sizes) >= 512 and max(nv for _, nv in sizes) >= 1024, sizes
    for o, r in zip(out, sorted(reqs, key=lambda r: r.rid)):
        # alone, cut into the scheduler's quanta of 7 steps
        s = vog.Sim(r.workload).init()
        left = r.workload.nsteps
        while left > 0:
            s.step(min(7, left))
            left -= min(7, left)
        assert np.array_equal(s.get_raw(), o.result["raw"]), r.rid
        assert np.array_equal(s.get_E(), o.result["E"]), r.rid
        s.close()


def test_diverged_request_fails_alone(gpu):
    from paper_1301_5892_amd import serving

    class NanExecutor(serving.GpuExecutor):
        def start(self, req):
            sim = super().start(req)
            if req.rid == 2:
                f = sim.get_f()
                f[3, 5] = float("nan")
                sim.set_f(f)
            return sim

    reqs = small_mix(6)
    ex = NanExecutor()
    out = serving.Scheduler(ex, budget_bytes=1 << 34, max_active=6, quantum=10).run(reqs)
    status = {o.rid: o.status for o in out}
    assert status[2] == "failed"
    assert all(s == "done" for rid, s in status.items() if rid != 2)


def test_serving_summary(gpu):
    from paper_1301_5892_amd import serving
    reqs = workloads.serving_mix(16, rate=200.0, seed=11, steps_range=(20, 40))
    out = serving.Scheduler(serving.GpuExecutor(), budget_bytes=1 << 34, max_active=8,
                            quantum=10).run(reqs)
    s = serving.summarize(out)
    assert s["done"] == 16
    assert 0 < s["p50_latency_s"] <= s["p99_latency_s"]
    assert s["aggregate_cell_updates_per_s"] > 0


def test_sync_batch_flags_only_the_diverged_sim(gpu):
    # 70 sims (two gather launches of at most 64); sim 66 gets a NaN in f.
    from paper_1301_5892_amd import vog
    base = workloads.landau_weak()
    sims = [vog.Sim(base.replace(nx=64, nv=128, amp=(0.01 + 1e-4 * i,))).init() for i in range(70)]
    assert vog.sync_batch(sims) == [True] * 70            # step 0: nothing recorded yet
    f = sims[66].get_f()
    f[3, 5] = float("nan")
    sims[66].set_f(f)
    vog.step_batch(sims, 2)
    ok = vog.sync_batch(sims)
    assert ok == [k != 66 for k in range(70)]
    for k in (0, 63, 64, 66, 69):                          # the single-sim call agrees
        if k == 66:
            with pytest.raises(vog.VogError):
                sims[k].sync()
        else:
            sims[k].sync()


def test_sync_batch_rejects_bad_arguments(gpu):
    import ctypes

    import torch

    from paper_1301_5892_amd import vog
    L = vog.load()
    a = vog.Sim(workloads.landau_weak()).init()
    st = (ctypes.c_int * 2)()
    one = (vog._P * 1)(a.handle)
    assert L.vog_sync_batch(one, 0, st) == vog.EINVAL
    assert L.vog_sync_batch(one, 1, None) == vog.EINVAL
    other = torch.cuda.Stream()
    b = vog.Sim(workloads.landau_weak(), stream=other).init()
    two = (vog._P * 2)(a.handle, b.handle)
    assert L.vog_sync_batch(two, 2, st) == vog.EINVAL     # different streams
    torch.cuda.synchronize()
