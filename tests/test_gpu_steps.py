"""Steps of one call against single-step calls (Section 1.1).

Inside one call of n steps the closing v half-step of each step and the
opening half-step of the next use the same field, and the library runs the
two in one launch.

With bitwise_steps (and for FP64 sims) each line pair is transformed twice,
the first result staged through LDS.  That changes where values live between
the two half-steps, not what is computed: f, E and every diagnostics record
must be bitwise those of n single-step calls, for every kernel family that
can take that launch (line lengths with several pairs per block, one wave per
pair and one pair per block; FP32 and FP64, delta f and plain; B-splines; the
KEEN drive; moments between steps; mixed-length batches).

By default FP32 sims compose the two half-steps in Fourier space (the symbol
applied twice, the first step's source transformed beside the lines, one
inverse transform): the same scheme with other rounding, so a call must stay
within the FP32 parity tolerance of single-step calls, and the same calls
must give the same bits alone and in a batch.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _run(gpu, w, split, moments_every=0, precision=None):
    s = gpu.Sim(w, moments_every=moments_every, precision=precision).init()
    for k in split:
        s.step(k)
    s.sync()
    return s.get_raw().copy(), s.get_E().copy(), s.diag().copy()


def _same(a, b):
    fa, ea, da = a
    fb, eb, db = b
    assert np.array_equal(fa, fb)
    assert np.array_equal(ea, eb)
    assert da.shape == db.shape
    assert da.tobytes() == db.tobytes()  # NaN-safe: the records' bytes


GRIDS = [
    ("fp32_deltaf", 64, 64),      # 8 line pairs per block, one wave per pair
    ("fp32_deltaf", 32, 1024),    # one wave per pair
    ("fp32_deltaf", 32, 2048),    # two pairs per block
    ("fp32_deltaf", 32, 4096),    # one pair per block
    ("fp32_plain", 64, 512),
    ("fp64_plain", 64, 256),
    ("fp64_deltaf", 32, 1024),
    ("fp64_plain", 32, 4096),     # two launches of the one-step kernel
]


@pytest.mark.parametrize("precision,nx,nv", GRIDS)
def test_call_equals_single_steps(gpu, precision, nx, nv):
    w = workloads.landau_strong().replace(nx=nx, nv=nv, precision=precision, bitwise_steps=True)
    _same(_run(gpu, w, [6]), _run(gpu, w, [1] * 6))


def test_call_chunks_equal(gpu):
    w = workloads.bump_on_tail().replace(nx=256, nv=512, bitwise_steps=True)
    ref = _run(gpu, w, [9])
    _same(ref, _run(gpu, w, [4, 5]))
    _same(ref, _run(gpu, w, [2, 1, 6]))


def test_moments_between_steps(gpu):
    # moments due after steps 2 and 4: those steps close with a single half step
    w = workloads.landau_strong().replace(nx=64, nv=256, bitwise_steps=True)
    a = _run(gpu, w, [5], moments_every=2)
    b = _run(gpu, w, [1] * 5, moments_every=2)
    _same(a, b)
    d = a[2]
    due = (d["step"] > 0) & (d["step"] % 2 == 0)
    assert due.sum() == 2 and np.isfinite(d["l2"][due]).all()


def test_bspline(gpu):
    w = workloads.landau_strong().replace(nx=64, nv=512, interp="bspline", degree=5, bitwise_steps=True)
    _same(_run(gpu, w, [5]), _run(gpu, w, [1] * 5))


def test_keen_drive(gpu):
    # the drive on from t = 0: the advecting field E - E_app differs from E
    d = workloads.Drive(t0=-60.0, tl=-50.0)
    w = workloads.keen(128, 0.1, 10).replace(drive=d, bitwise_steps=True)
    _same(_run(gpu, w, [6]), _run(gpu, w, [1] * 6))


def test_mixed_batch_call_equals_single_steps(gpu):
    from paper_1301_5892_amd import vog
    ws = [workloads.landau_strong().replace(nx=64, nv=n, bitwise_steps=True) for n in (128, 1024, 4096)]
    ws.append(workloads.landau_weak().replace(nx=128, nv=256))
    alone = [_run(gpu, w, [1] * 4) for w in ws]
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 4)
    for s, a in zip(sims, alone):
        s.sync()
        _same((s.get_raw(), s.get_E(), s.diag()), a)


def test_batch_of_130_mixed_lengths(gpu):
    # More sims than one launch of 64, and than one sweep launch of 128: the
    # sweeps' launch table (two ballots per wave) and the chunking at 128,
    # the field solves' chunking at 64.
    from paper_1301_5892_amd import vog
    rng = np.random.default_rng(5)
    ws = []
    for k in range(130):
        nx = int(2 ** rng.integers(5, 8))     # 32 .. 128
        nv = int(2 ** rng.integers(6, 10))    # 64 .. 512
        ws.append(workloads.landau_strong().replace(nx=nx, nv=nv, amp=(0.05 + 0.003 * k,)))
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 3)
    for s in sims:
        s.sync()
    for k in (0, 63, 64, 65, 100, 127, 128, 129):
        a = _run(gpu, ws[k], [3])
        _same((sims[k].get_raw(), sims[k].get_E(), sims[k].diag()), a)


# ------------------------------------------------- composed (the default, FP32)

TOL32 = 1e-5  # the FP32 parity tolerance, relative to the array's largest value


def _close(a, b, tol=TOL32):
    for x, y in zip(a[:2], b[:2]):
        x, y = x.astype(np.float64), y.astype(np.float64)
        assert np.isfinite(x).all()
        assert np.max(np.abs(x - y)) <= tol * np.max(np.abs(y))
    assert np.array_equal(a[2]["step"], b[2]["step"])


COMPOSED = [
    ("fp32_deltaf", 64, 8, 7),     # one thread per pair, radix-8 transform
    ("fp32_deltaf", 64, 16, 9),    # one thread per pair (no LDS exchange)
    ("fp32_plain", 64, 32, 17),    # two threads per pair, one exchange
    ("fp32_deltaf", 64, 64, 17),   # 8 line pairs per block
    ("fp32_deltaf", 32, 1024, 17), # one wave per pair
    ("fp32_deltaf", 32, 2048, 17), # two pairs per block
    ("fp32_deltaf", 32, 4096, 17), # one pair per block
    ("fp32_plain", 64, 512, 17),
    ("fp32_plain", 32, 4096, 17),
]


@pytest.mark.parametrize("precision,nx,nv,degree", COMPOSED)
def test_composed_call_close_to_single_steps(gpu, precision, nx, nv, degree):
    w = workloads.landau_strong().replace(nx=nx, nv=nv, precision=precision, degree=degree)
    one = _run(gpu, w, [6])
    _close(one, _run(gpu, w, [1] * 6))
    _same(one, _run(gpu, w, [6]))  # the same calls, the same bits


def test_composed_differs_from_bitwise(gpu):
    # the composed launch is the one that runs by default
    w = workloads.landau_strong().replace(nx=64, nv=1024)
    a, b = _run(gpu, w, [6]), _run(gpu, w.replace(bitwise_steps=True), [6])
    _close(a, b)
    assert not np.array_equal(a[0], b[0])


def test_composed_bspline_and_drive(gpu):
    w = workloads.landau_strong().replace(nx=64, nv=512, interp="bspline", degree=5)
    _close(_run(gpu, w, [5]), _run(gpu, w, [1] * 5))
    d = workloads.Drive(t0=-60.0, tl=-50.0)
    w = workloads.keen(128, 0.1, 10).replace(drive=d)
    _close(_run(gpu, w, [6]), _run(gpu, w, [1] * 6))


def test_composed_moments_between_steps(gpu):
    w = workloads.landau_strong().replace(nx=64, nv=256)
    a = _run(gpu, w, [5], moments_every=2)
    _close(a, _run(gpu, w, [1] * 5, moments_every=2))
    d = a[2]
    due = (d["step"] > 0) & (d["step"] % 2 == 0)
    assert due.sum() == 2 and np.isfinite(d["l2"][due]).all()


def test_composed_mixed_batch_equals_alone(gpu):
    # the mixed-length launch and the single-length one run the same body
    from paper_1301_5892_amd import vog
    ws = [workloads.landau_strong().replace(nx=64, nv=n) for n in (128, 1024, 4096)]
    ws.append(workloads.landau_strong().replace(nx=128, nv=256, precision="fp32_plain"))
    alone = [_run(gpu, w, [4]) for w in ws]
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 4)
    for s, a in zip(sims, alone):
        s.sync()
        _same((s.get_raw(), s.get_E(), s.diag()), a)
