"""vog_sync_batch_noalloc (no device allocation, flags in the library's fixed
device array) through the C ABI against vog_sync_batch on the same sims: two
calls in a row, the second with fewer sims, each with sims whose field is not
finite (a NaN planted in f from the host) among finite ones."""
import ctypes

import pytest

import workloads

pytestmark = pytest.mark.gpu


def _both(L, vog, sims):
    n = len(sims)
    arr = (vog._P * n)(*[s.handle for s in sims])
    ref = (ctypes.c_int * n)()
    got = (ctypes.c_int * n)(*([12345] * n))  # every entry must be overwritten
    assert L.vog_sync_batch(arr, n, ref) == vog.OK
    assert L.vog_sync_batch_noalloc(arr, n, got) == vog.OK
    return list(ref), list(got)


def test_noalloc_sync_batch_equals_sync_batch(gpu):
    vog = gpu
    L = vog.load()
    base = workloads.landau_weak()
    # 70 sims: two gathers of at most 64 into the fixed array
    sims = [vog.Sim(base.replace(nx=64, nv=128, amp=(0.01 + 1e-4 * i,))).init() for i in range(70)]
    bad = {3, 64, 66}
    for k in bad:
        f = sims[k].get_f()
        f[5, 7] = float("nan")
        sims[k].set_f(f)
    vog.step_batch(sims, 2)
    ref, got = _both(L, vog, sims)
    assert got == ref
    assert got == [vog.ENONFINITE if k in bad else vog.OK for k in range(70)]

    # second call, fewer sims and a different pattern: sims 0..9, of which 3 diverged
    few = sims[:10]
    f = few[8].get_f()
    f[1, 2] = float("inf")
    few[8].set_f(f)
    vog.step_batch(few, 1)
    ref2, got2 = _both(L, vog, few)
    assert got2 == ref2
    assert got2 == [vog.ENONFINITE if k in (3, 8) else vog.OK for k in range(10)]


def test_noalloc_sync_batch_rejects_bad_arguments(gpu):
    vog = gpu
    L = vog.load()
    a = vog.Sim(workloads.landau_weak()).init()
    st = (ctypes.c_int * 2)()
    one = (vog._P * 1)(a.handle)
    assert L.vog_sync_batch_noalloc(one, 0, st) == vog.EINVAL
    assert L.vog_sync_batch_noalloc(one, 1, None) == vog.EINVAL
    assert L.vog_sync_batch_noalloc(None, 1, st) == vog.EINVAL
    n = vog.NOALLOC_MAX_SIMS + 1
    many = (vog._P * n)(*([a.handle] * n))
    big = (ctypes.c_int * n)()
    assert L.vog_sync_batch_noalloc(many, n, big) == vog.EINVAL
