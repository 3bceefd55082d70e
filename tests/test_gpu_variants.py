"""GPU parity of the method's variants against the CPU FP64 oracle, through
the C ABI: B-spline interpolation (Section 1.2), merged v half-steps
(Section 1.1), single precision without the delta-f split (Section 4.1),
and the paper's single-precision study (Section 4.1), which compares how
long each variant follows weak Landau damping.

Tolerances as in the other parity tests: 1e-12 relative for FP64, 1e-5 for
FP32 (on delta f, or on f for the plain FP32 variant).
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
TOL64_E = 1e-11  # FP64 E and ||E||_2 after several steps (see test_gpu_parity.TOL64_E)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel_field(E, o):
    """E error relative to (L / 2 pi) max|rho|: only for driven runs from
    f = f_M, whose self-consistent E starts at rounding level (see
    test_gpu_parity.rel_field)."""
    scale = max(np.max(np.abs(o.E)), o.w.L / (2 * math.pi) * np.max(np.abs(o.rho)))
    return float(np.max(np.abs(np.asarray(E) - o.E)) / scale)


def spline(w, k=3):
    return w.replace(interp="bspline", degree=k)


# ---------------------------------------------------------------- B-spline sweeps

# Both x-sweep layouts (tiled for nx >= 256 with enough v-rows, transposed
# otherwise), line lengths 8 .. 2048, degrees 1 .. 17.
BSPLINE_GRIDS = [(8, 8, 3), (16, 32, 5), (64, 128, 3), (256, 64, 3), (512, 256, 17),
                 (1024, 64, 3), (128, 1024, 7), (2048, 16, 3), (32, 32, 1), (256, 512, 9)]


@pytest.mark.parametrize("nx,nv,k", BSPLINE_GRIDS, ids=lambda x: str(x))
@pytest.mark.parametrize("dt", [0.1, -2.3])
def test_bspline_x_sweep_fp64(gpu, nx, nv, k, dt):
    w = spline(workloads.landau_weak().replace(nx=nx, nv=nv, amp=(0.3, 0.1), kx=(0.5, 1.5),
                                                phase=(0.2, 1.0)), k)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.advect_x(dt)
    o.advect_x(dt)
    assert rel(s.get_f(), o.f) < TOL64


@pytest.mark.parametrize("nx,nv,k", BSPLINE_GRIDS, ids=lambda x: str(x))
@pytest.mark.parametrize("precision", ["fp64_plain", "fp64_deltaf"])
def test_bspline_v_sweep_fp64(gpu, nx, nv, k, precision):
    w = spline(workloads.landau_weak().replace(nx=nx, nv=nv, precision=precision, amp=(0.2,),
                                                kx=(0.5,), phase=(0.0,)), k)
    E = np.random.default_rng(nx + 3 * nv).uniform(-3.0, 3.0, nx)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.set_E(E)
    s.advect_v(0.35)
    o.advect_v(0.35, E)
    assert rel(s.get_raw(), o.f) < TOL64


@pytest.mark.parametrize("nx,nv,k", [(64, 128, 3), (256, 512, 3), (1024, 64, 5), (512, 2048, 3)])
def test_bspline_sweeps_fp32_deltaf(gpu, nx, nv, k):
    w = spline(workloads.landau_strong().replace(nx=nx, nv=nv, amp=(0.3, 0.1), kx=(0.5, 1.5),
                                                  phase=(0.2, 1.0)), k)
    E = np.random.default_rng(11).uniform(-1.5, 1.5, nx)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.advect_x(0.7)
    o.advect_x(0.7)
    assert rel(s.get_raw(), o.f) < TOL32
    s.set_E(E)
    o.E = E.copy()
    s.advect_v(0.25)
    o.advect_v(0.25, E)
    assert rel(s.get_raw(), o.f) < TOL32


@pytest.mark.parametrize("n", [4096, 256])
@pytest.mark.parametrize("precision", ["fp64_plain", "fp32_deltaf"])
def test_bspline_integer_shift_is_roll(gpu, n, precision):
    # A spline interpolates its data, so an integer shift returns it exactly
    # up to rounding, at any size (here the full 4096-point lines).
    w = spline(workloads.landau_strong().replace(nx=64, nv=n, precision=precision,
                                                  amp=(0.3,), kx=(0.5,), phase=(0.0,)), 3)
    s = gpu.Sim(w).init()
    f0 = s.get_raw().astype(np.float64)
    dv = (w.vmax - w.vmin) / w.nv
    E = np.full(w.nx, -3.0 * dv / 0.5)  # beta = 3 cells along the n-point v-lines
    s.set_E(E)
    s.advect_v(0.5)
    got = s.get_raw().astype(np.float64)
    if precision == "fp32_deltaf":
        # delta-f adds f_eq(v - tau E) - f_eq(v) = f_eq(v_{j+3}) - f_eq(v_j)
        o = oracle.Oracle(w)
        feq = o.feq_grid()
        ref = np.roll(f0, -3, axis=1) + (np.roll(feq, -3) - feq)[None, :]
        assert rel(got, ref) < TOL32
    else:
        assert rel(got, np.roll(f0, -3, axis=1)) < TOL64


def test_bspline_landau_run_fp64(gpu):
    w = spline(workloads.landau_weak(), 3)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(30)
    od = o.step(30)
    assert rel(s.get_f(), o.f) < TOL64
    assert rel(s.get_E(), o.E) < TOL64_E
    d = s.diag()
    assert np.max(np.abs(d["normE"][1:] - od[:, 0]) / od[:, 0]) < TOL64_E


@pytest.mark.parametrize("k", [3, 5])
def test_bspline_strong_run_fp32(gpu, k):
    w = spline(workloads.landau_strong(), k)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(10)
    o.step(10)
    assert rel(s.get_raw(), o.f) < TOL32
    assert rel(s.get_E(), o.E) < TOL32


def test_bspline_keen_fp32(gpu):
    d = workloads.Drive(t0=-60.0, tl=-50.0)
    w = spline(workloads.keen(256, 0.1, 10).replace(drive=d), 3)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(10)
    o.step(10)
    assert rel(s.get_raw(), o.f) < TOL32
    assert rel(s.get_E(), o.E) < TOL32


# ---------------------------------------------------------------- merged v half-steps

def merged(w):
    return w.replace(merge_v=True)


def test_merged_landau_fp64(gpu):
    w = merged(workloads.landau_weak())
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(w.nsteps)
    od = o.step(w.nsteps)
    assert rel(s.get_f(), o.f) < TOL64
    assert rel(s.get_E(), o.E) < TOL64_E
    d = s.diag()
    assert np.max(np.abs(d["normE"][1:] - od[:, 0]) / od[:, 0]) < TOL64_E


def test_merged_strong_fp32(gpu):
    w = merged(workloads.landau_strong())
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(10)
    o.step(10)
    assert rel(s.get_raw(), o.f) < TOL32
    assert rel(s.get_E(), o.E) < TOL32


def test_merged_keen_fp64(gpu):
    d = workloads.Drive(t0=-60.0, tl=-50.0)
    w = merged(workloads.keen(64, 0.1, 20).replace(precision="fp64_plain", drive=d))
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(20)
    o.step(20)
    assert rel(s.get_f(), o.f) < TOL64
    assert rel_field(s.get_E(), o) < TOL64


def test_merged_calls_close_with_half_steps(gpu):
    # Each call starts and ends with a half step: two calls of 5 steps equal
    # the oracle's two runs of 5, and differ from one call of 10.
    w = merged(workloads.landau_weak())
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(5)
    s.step(5)
    o.step(5)
    o.step(5)
    assert rel(s.get_f(), o.f) < TOL64
    one = gpu.Sim(w).init()
    one.step(10)
    assert not np.array_equal(one.get_f(), s.get_f())


def test_merged_batch_equals_alone(gpu):
    from paper_1301_5892_amd import vog
    ws = [merged(workloads.landau_weak()), workloads.landau_weak(),
          merged(workloads.landau_strong())]
    alone = []
    for w in ws:
        s = gpu.Sim(w).init()
        s.step(7)
        alone.append(s.get_raw())
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 7)
    for s, a in zip(sims, alone):
        assert np.array_equal(s.get_raw(), a)


def test_merged_moments_only_at_full_levels(gpu):
    w = merged(workloads.landau_weak())
    s = gpu.Sim(w, moments_every=1).init()
    s.step(6)
    d = s.diag()
    rec = d[d["step"] > 0]
    assert np.all(np.isnan(rec["l2"][:-1])) and np.isfinite(rec["l2"][-1])


# ---------------------------------------------------------------- FP32 without delta f

@pytest.mark.parametrize("nx,nv", [(64, 128), (256, 512), (1024, 64), (32, 4096)])
def test_fp32_plain_sweeps(gpu, nx, nv):
    w = workloads.landau_strong().replace(nx=nx, nv=nv, precision="fp32_plain",
                                           degree=min(17, nv - 1))
    E = np.random.default_rng(2).uniform(-1.5, 1.5, nx)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    assert not o.deltaf
    s.advect_x(0.9)
    o.advect_x(0.9)
    assert rel(s.get_raw(), o.f) < TOL32
    s.set_E(E)
    s.advect_v(0.25)
    o.advect_v(0.25, E)
    assert rel(s.get_raw(), o.f) < TOL32


@pytest.mark.parametrize("poisson,zero_mean", [("fourier", True), ("trapezoid", True),
                                               ("trapezoid", False)])
def test_fp32_plain_runs(gpu, poisson, zero_mean):
    w = workloads.landau_strong().replace(precision="fp32_plain", poisson=poisson,
                                           zero_mean=zero_mean)
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(10)
    o.step(10)
    assert rel(s.get_raw(), o.f) < TOL32
    assert rel(s.get_E(), o.E) < TOL32


# ---------------------------------------------------------------- precision study (Section 4.1)

def _departure(gpu, w, precision, poisson="fourier", zero_mean=True, ref=None):
    """||E||_2 history of weak Landau damping, and the first time at which
    it leaves the FP64 history by more than a factor 2 (the end time if it
    never does)."""
    w = w.replace(precision=precision, poisson=poisson, zero_mean=zero_mean)
    s = gpu.Sim(w).init()
    s.step(w.nsteps)
    e = s.diag()["normE"][1:]
    s.close()
    if ref is None:
        return e, None
    with np.errstate(all="ignore"):
        bad = np.nonzero(~(np.abs(np.log(e / ref)) <= math.log(2.0)))[0]
    t = (bad[0] + 1) * w.dt if bad.size else w.nsteps * w.dt
    return e, t


def test_single_precision_study(gpu, capsys):
    # Section 4.1 (LAG17, N = 2048, v in [-8, 8)): in single precision the
    # delta-f form follows the damping longest; without it the zero-mean
    # solves (Fourier, trapezoid with zero mean) come next; the trapezoidal
    # solve without the zero-mean step saturates first.
    w = workloads.landau_weak().replace(nx=2048, nv=2048, vmin=-8.0, vmax=8.0, nsteps=600)
    ref, _ = _departure(gpu, w, "fp64_plain")
    assert np.all(np.isfinite(ref))
    _, t_df = _departure(gpu, w, "fp32_deltaf", ref=ref)
    _, t_fourier = _departure(gpu, w, "fp32_plain", ref=ref)
    _, t_trap_zm = _departure(gpu, w, "fp32_plain", "trapezoid", True, ref=ref)
    _, t_trap = _departure(gpu, w, "fp32_plain", "trapezoid", False, ref=ref)
    with capsys.disabled():
        print(f"\nsingle-precision study, time at which ||E|| leaves FP64 by 2x: "
              f"delta-f {t_df:.1f}, plain Fourier {t_fourier:.1f}, plain trapezoid "
              f"zero-mean {t_trap_zm:.1f}, plain trapezoid {t_trap:.1f}")
    assert t_df > t_fourier
    assert t_df > t_trap_zm
    assert t_trap < min(t_fourier, t_trap_zm)


# ---------------------------------------------------------------- edge cases

def test_zero_steps_is_a_no_op(gpu):
    w = workloads.landau_strong()
    s = gpu.Sim(w).init()
    f0 = s.get_raw().copy()
    s.diag()
    s.step(0)
    assert np.array_equal(s.get_raw(), f0)
    assert s.diag().size == 0
    assert s.time() == (0, 0.0)


def test_batch_arguments_rejected(gpu):
    import ctypes
    from paper_1301_5892_amd import vog
    L = vog.load()
    s = gpu.Sim(workloads.landau_weak()).init()
    dt = (ctypes.c_double * 2)(0.1, 0.1)
    one = (ctypes.c_void_p * 1)(s.handle)
    assert L.vog_step_batch(one, 0, dt, 1) == vog.EINVAL
    two = (ctypes.c_void_p * 2)(s.handle, s.handle)
    assert L.vog_step_batch(two, 2, dt, 1) == vog.EINVAL    # same sim twice
    assert L.vog_step_batch(one, 1, dt, -1) == vog.EINVAL
    bad = (ctypes.c_double * 1)(-0.1)
    assert L.vog_step_batch(one, 1, bad, 1) == vog.EINVAL


@pytest.mark.parametrize("interp,k", [("lagrange", 7), ("bspline", 7), ("bspline", 1)])
@pytest.mark.parametrize("precision,tol", [("fp64_plain", TOL64), ("fp32_deltaf", TOL32)])
def test_smallest_grid_runs(gpu, interp, k, precision, tol):
    # 8 x 8, the smallest grid, with the widest stencil it allows.
    w = workloads.landau_weak().replace(nx=8, nv=8, degree=k, interp=interp, precision=precision,
                                         amp=(0.3,), kx=(0.5,), phase=(0.1,))
    s = gpu.Sim(w).init()
    o = oracle.Oracle(w).init()
    s.step(5)
    o.step(5)
    got = s.get_raw() if precision == "fp32_deltaf" else s.get_f()
    assert rel(got, o.f) < tol


def test_diag_ring_wraps(gpu):
    # Records are read in pieces that straddle the end of the 4096-record ring.
    w = workloads.landau_weak().replace(nx=8, nv=8, degree=7)
    s = gpu.Sim(w).init()
    s.step(4090)
    d0 = s.diag()
    assert d0["step"][-1] == 4090 and np.all(np.diff(d0["step"]) == 1)
    s.step(20)
    d1 = s.diag()
    assert list(d1["step"]) == list(range(4091, 4111))
    assert np.all(d1["finite"] == 1)
    ref = gpu.Sim(w).init()
    ref.step(4110)
    r = ref.diag()
    assert np.array_equal(r["normE"][-20:], d1["normE"])


def test_bump_on_tail_mass_error_ordering(gpu, capsys):
    # Section 4.2 (bump on tail): the mass error |rho_hat_0(t) - rho_hat_0(0)|
    # accumulates in time; in single precision the delta-f form keeps it
    # smaller than plain f, and double precision is far below both.
    w = workloads.bump_on_tail().replace(nsteps=2000)
    err = {}
    for precision in ("fp64_plain", "fp32_deltaf", "fp32_plain"):
        s = gpu.Sim(w.replace(precision=precision)).init()
        s.step(w.nsteps)
        d = s.diag()
        s.close()
        assert np.all(d["finite"] == 1)
        drift = np.abs(d["rho0"] - d["rho0"][0])
        err[precision] = (float(np.max(drift[: w.nsteps // 4 + 1])), float(np.max(drift)))
    with capsys.disabled():
        print("\nbump-on-tail mass error (first quarter, whole run): " +
              ", ".join(f"{k} {a:.2e} {b:.2e}" for k, (a, b) in err.items()))
    assert err["fp64_plain"][1] < 1e-3 * err["fp32_deltaf"][1]
    assert err["fp32_deltaf"][1] < err["fp32_plain"][1]
    for k in ("fp32_deltaf", "fp32_plain"):
        assert err[k][1] > err[k][0]          # it accumulates


# ---------------------------------------------------------------- mixed line lengths

# FP32 sims whose lines differ in length share one sweep launch per phase (every
# v-line length from 64 to 4096 points, x-lines from 64 to 1024 points on the
# v-fastest layout).  Each sim must come out exactly as when stepped alone.
def _mixed_fp32():
    base = workloads.landau_weak()
    return [base.replace(nx=64, nv=4096, precision="fp32_deltaf"),
            base.replace(nx=1024, nv=128, precision="fp32_deltaf"),
            base.replace(nx=128, nv=2048, precision="fp32_deltaf"),
            base.replace(nx=256, nv=256, precision="fp32_deltaf"),
            base.replace(nx=512, nv=512, precision="fp32_deltaf"),
            # (FP32 without delta f at a strong amplitude: rho - mean(rho) well
            # above the rounding of f stored in FP32)
            base.replace(nx=64, nv=128, precision="fp32_plain", amp=(0.5,)),
            spline(base.replace(nx=128, nv=1024, precision="fp32_deltaf"), 5),
            base.replace(nx=32, nv=64, precision="fp32_deltaf"),
            # v-lines of 32 points: their own launch beside the mixed one
            base.replace(nx=64, nv=32, precision="fp32_deltaf")]


def test_mixed_lengths_batch_equals_alone(gpu):
    from paper_1301_5892_amd import vog
    ws = _mixed_fp32()
    alone = []
    for w in ws:
        s = gpu.Sim(w).init()
        s.step(6)
        alone.append((s.get_raw(), s.get_E()))
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 6)
    for w, s, (f0, e0) in zip(ws, sims, alone):
        assert np.array_equal(s.get_raw(), f0), w.name
        assert np.array_equal(s.get_E(), e0), w.name


def test_mixed_lengths_batch_matches_oracle(gpu):
    from paper_1301_5892_amd import vog
    ws = _mixed_fp32()
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 3)
    for w, s in zip(ws, sims):
        o = oracle.Oracle(w).init()
        o.step(3)
        # stored arrays: delta f for the delta-f variants, f for plain FP32
        assert rel(s.get_raw(), o.f) < TOL32, w.name
        assert rel(s.get_E(), o.E) < TOL32, w.name


def test_mixed_lengths_more_sims_than_one_launch(gpu):
    # 72 sims: the mixed launches split into chunks of at most 64 sims.
    from paper_1301_5892_amd import vog
    base = workloads.landau_weak()
    sizes = [(64, 128), (128, 256), (64, 512), (256, 128)]
    ws = [base.replace(nx=sizes[i % 4][0], nv=sizes[i % 4][1], precision="fp32_deltaf",
                       amp=(0.01 + 0.001 * i,)) for i in range(72)]
    alone = []
    for w in ws[:4] + ws[-4:]:
        s = gpu.Sim(w).init()
        s.step(4)
        alone.append(s.get_raw())
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 4)
    for s, f0 in zip(sims[:4] + sims[-4:], alone):
        assert np.array_equal(s.get_raw(), f0)


def test_mixed_lengths_with_merged_and_driven_sims(gpu):
    # A batch that mixes line lengths, merged v half-steps, a KEEN-driven sim,
    # FP64 sims (their own kernels) and nx < 64 (transposed x-sweep): each
    # sim equals the same sim stepped alone, over two calls.
    from paper_1301_5892_amd import vog
    base = workloads.landau_weak()
    ws = [merged(base.replace(nx=256, nv=512, precision="fp32_deltaf")),
          base.replace(nx=128, nv=1024, precision="fp32_deltaf"),
          workloads.keen(128, 0.1, 20).replace(nv=256),
          base.replace(nx=512, nv=128, precision="fp64_plain"),
          base.replace(nx=32, nv=256, precision="fp32_deltaf"),
          merged(base.replace(nx=64, nv=2048, precision="fp32_plain"))]
    alone = []
    for w in ws:
        s = gpu.Sim(w).init()
        s.step(5)
        s.step(4)
        alone.append((s.get_raw(), s.get_E()))
    sims = [gpu.Sim(w).init() for w in ws]
    vog.step_batch(sims, 5)
    vog.step_batch(sims, 4)
    for w, s, (f0, e0) in zip(ws, sims, alone):
        assert np.array_equal(s.get_raw(), f0), w.name
        assert np.array_equal(s.get_E(), e0), w.name
