"""Pins of the CPU FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: algebraic
identities of Lagrange interpolation, exact integer shifts, exact translation
of resolved Fourier modes, closed-form Poisson solutions, the free-streaming
exact solution, conservation laws, the paper's Landau damping rate and
oscillation counts, and second-order convergence of the Strang splitting.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1234)


# ------------------------------------------------------------------ weights

@pytest.mark.parametrize("d", [0, 1, 4, 8])
def test_weights_partition_of_unity(orc, d):
    for s in RNG.uniform(0, 1, 20):
        assert abs(orc.lagrange_weights(d, s).sum() - 1.0) < 1e-13


@pytest.mark.parametrize("d", [1, 4, 8])
def test_weights_reproduce_polynomials(orc, d):
    # Lagrange interpolation on nodes -d..d+1 is exact for degree <= 2d+1:
    # sum_q w_q(s) p(q) = p(s).
    q = np.arange(-d, d + 2)
    for s in RNG.uniform(0, 1, 10):
        w = orc.lagrange_weights(d, s)
        for k in range(2 * d + 2):
            p = lambda x: ((x - 0.5) / (d + 1)) ** k
            assert abs(np.dot(w, p(q)) - p(s)) < 1e-13


@pytest.mark.parametrize("d", [1, 4, 8])
def test_weights_not_exact_beyond_degree(orc, d):
    # Degree 2d+2 is not reproduced (guards against a dropped node).
    q = np.arange(-d, d + 2)
    w = orc.lagrange_weights(d, 0.37)
    p = lambda x: ((x - 0.5) / (d + 1)) ** (2 * d + 2)
    assert abs(np.dot(w, p(q)) - p(0.37)) > 1e-10


@pytest.mark.parametrize("d", [0, 1, 4, 8])
def test_weights_mirror_symmetry(orc, d):
    # w_q(s) = w_{1-q}(1-s): the stencil is centred on the cell of the foot.
    for s in RNG.uniform(0, 1, 5):
        w = orc.lagrange_weights(d, s)
        wm = orc.lagrange_weights(d, 1.0 - s)
        assert np.allclose(w, wm[::-1], rtol=0, atol=1e-14)


def test_lagrange1_closed_form(orc):
    # Section 1.2, Lagrange 1: a_b = 1 - b*, a_{b+1} = b*.
    for s in RNG.uniform(0, 1, 10):
        assert np.allclose(orc.lagrange_weights(0, s), [1.0 - s, s], atol=1e-15)


@pytest.mark.parametrize("d", [0, 4, 8])
def test_weights_at_zero_shift(orc, d):
    w = orc.lagrange_weights(d, 0.0)
    e = np.zeros(2 * d + 2)
    e[d] = 1.0
    assert np.array_equal(w, e)


def test_split_shift(orc):
    for beta in [0.0, 0.25, -0.25, 3.0, -3.0, 52.7, -52.7, 1e-17, -1e-17, 7.999999999]:
        b, s = orc.split_shift(beta)
        assert isinstance(b, int) and 0.0 <= s < 1.0
        assert abs((b + s) - beta) <= 1e-15 * max(1.0, abs(beta))


# ------------------------------------------------------------------ one line

@pytest.mark.parametrize("beta", [0, 1, -1, 5, -17, 64, 131, -200])
def test_integer_shift_is_exact_roll(orc, beta):
    n = 64
    u = RNG.standard_normal(n)
    out = orc.advect_line(u, 8, float(beta))
    # out_i = u_{(i + beta) mod n}
    assert np.array_equal(out, np.roll(u, -beta))


@pytest.mark.parametrize("beta", [0.3, 2.71, -4.45, -0.999])
def test_polynomial_reproduction_interior(orc, beta):
    d, n = 8, 128
    coef = RNG.standard_normal(2 * d + 2)
    p = lambda x: np.polyval(coef, (x - n / 2) / n)
    i = np.arange(n)
    out = orc.advect_line(p(i.astype(float)), d, beta)
    b = math.floor(beta)
    interior = (i + b - d >= 0) & (i + b + d + 1 <= n - 1)
    assert interior.sum() > 60
    assert np.max(np.abs(out[interior] - p(i[interior] + beta))) < 1e-12


@pytest.mark.parametrize("m", [1, 2, 3])
def test_resolved_mode_is_translated(orc, m):
    # A resolved periodic mode is translated exactly up to the degree-17
    # interpolation error, which is far below FP64 rounding here.
    n = 256
    i = np.arange(n)
    th = 2 * math.pi * m / n
    for beta in [0.4, -3.3, 40.6]:
        out = orc.advect_line(np.cos(th * i + 0.2), 8, beta)
        assert np.max(np.abs(out - np.cos(th * (i + beta) + 0.2))) < 1e-13


@pytest.mark.parametrize("n,d", [(32, 8), (16, 4), (8, 1), (8, 0)])
def test_dense_circulant_matches_stencil(orc, n, d):
    # A = C(a_0 .. a_{n-1}): row i is the first row shifted right by i
    # (Section 1.2), so A[i, k] = a[(k - i) mod n].
    for beta in [0.37, -2.5, 9.99, -13.01]:
        a = orc.circulant_row(n, d, beta)
        A = np.array([[a[(k - i) % n] for k in range(n)] for i in range(n)])
        u = RNG.standard_normal(n)
        assert np.allclose(A @ u, orc.advect_line(u, d, beta), rtol=0, atol=1e-13)
        assert np.count_nonzero(a) == 2 * d + 2 or beta == round(beta)


# ------------------------------------------------------------------ field

def test_poisson_closed_form(orc):
    # dE/dx = rho - mean(rho); rho = 1 + a cos(k x) + c sin(3 k x)
    # gives E = (a/k) sin(k x) - c/(3k) cos(3 k x).
    w = workloads.landau_weak()
    o = orc.Oracle(w)
    x = o.x()
    k = 0.5
    rho = 1.0 + 0.3 * np.cos(k * x) + 0.05 * np.sin(3 * k * x)
    E = o.poisson(rho)
    ex = 0.3 / k * np.sin(k * x) - 0.05 / (3 * k) * np.cos(3 * k * x)
    assert np.max(np.abs(E - ex)) < 1e-13
    assert abs(E.mean()) < 1e-15


def test_poisson_drops_mean_and_nyquist(orc):
    w = workloads.landau_weak()
    o = orc.Oracle(w)
    rho = 3.0 + (-1.0) ** np.arange(w.nx)   # mean plus Nyquist only
    assert np.max(np.abs(o.poisson(rho))) < 1e-13


def test_rho_of_maxwellian_product(orc):
    # int f_M dv = 1 up to the Gaussian tail beyond |v| = 6 (< 2e-9) and the
    # spectrally small rectangle-rule error.
    w = workloads.landau_weak()
    o = orc.Oracle(w).init()
    x = o.x()
    assert np.max(np.abs(o.rho - (1.0 + 0.01 * np.cos(0.5 * x)))) < 5e-9


# ------------------------------------------------------------------ 2D runs

def test_free_streaming_exact(orc):
    w = workloads.free_streaming(64, 64, 20)
    o = orc.Oracle(w).init()
    o.step(w.nsteps)
    x, v = o.x()[:, None], o.v()[None, :]
    t = w.nsteps * w.dt
    fm = np.exp(-v ** 2 / 2) / math.sqrt(2 * math.pi)
    exact = (1 + 0.05 * np.cos(0.5 * (x - v * t) + 0.3)) * fm
    assert np.max(np.abs(o.full_f() - exact)) < 1e-13


def test_free_streaming_exact_deltaf(orc):
    w = workloads.free_streaming(64, 64, 20).replace(precision="fp64_deltaf")
    o = orc.Oracle(w).init()
    o.step(w.nsteps)
    x, v = o.x()[:, None], o.v()[None, :]
    t = w.nsteps * w.dt
    fm = np.exp(-v ** 2 / 2) / math.sqrt(2 * math.pi)
    assert np.max(np.abs(o.f - 0.05 * np.cos(0.5 * (x - v * t) + 0.3) * fm)) < 1e-14


def test_mass_conserved_plain(orc):
    w = workloads.landau_strong().replace(nx=64, nv=128, precision="fp64_plain")
    o = orc.Oracle(w).init()
    m0 = o.f.sum()
    o.step(20)
    assert abs(o.f.sum() - m0) / abs(m0) < 1e-13


def test_vadvect_deltaf_source_of_zero_perturbation(orc):
    # delta f = 0 and a field E: the update is f_eq(v - tau E) - f_eq(v)
    # exactly (Section 3.1, the evaluation term).
    w = workloads.landau_weak().replace(precision="fp64_deltaf")
    o = orc.Oracle(w)
    E = 0.3 * np.sin(o.x())
    tau = 0.05
    o.advect_v(tau, E)
    v = o.v()[None, :]
    fm = lambda vv: np.exp(-vv ** 2 / 2) / math.sqrt(2 * math.pi)
    assert np.max(np.abs(o.f - (fm(v - tau * E[:, None]) - fm(v)))) < 1e-15


def test_plain_and_deltaf_agree(orc):
    # Same physics in both forms; they differ by the interpolation error of
    # f_eq and its periodic seam, both tiny at |v| = 6.
    w = workloads.landau_weak()
    a = orc.Oracle(w, deltaf=False).init()
    b = orc.Oracle(w, deltaf=True).init()
    a.step(10)
    b.step(10)
    fa, fb = a.full_f(), b.full_f()
    assert np.max(np.abs(fa - fb)) / np.max(np.abs(fa)) < 1e-8
    assert np.max(np.abs(a.E - b.E)) / np.max(np.abs(a.E)) < 1e-6


def test_strang_is_second_order(orc):
    # Error at fixed t against a fine-dt run shrinks ~4x per halving of dt;
    # a first-order (Lie) ordering of the substeps would give ~2x.
    base = workloads.landau_strong().replace(nx=32, nv=64, vmin=-6.0, vmax=6.0,
                                             precision="fp64_plain")
    T = 1.6

    def run(dt):
        o = orc.Oracle(base.replace(dt=dt)).init()
        o.step(int(round(T / dt)))
        return o.f.copy()

    ref = run(0.0125)
    e = [np.max(np.abs(run(dt) - ref)) for dt in (0.2, 0.1, 0.05)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r1 < 4.8 and 3.3 < r2 < 4.8, (e, r1, r2)


def _paper():
    with open(os.path.join(GOLDEN, "landau_paper.json")) as fh:
        return json.load(fh)


def test_landau_weak_rate(orc):
    # Short run (t <= 10): rate within 5 % of the paper's value.
    w = workloads.landau_weak()
    o = orc.Oracle(w).init()
    d = o.step(w.nsteps)
    t = (np.arange(w.nsteps) + 1) * w.dt
    gamma, omega, _ = orc.landau_fit(t, d[:, 0])
    assert abs(-gamma - _paper()["gamma"]) / _paper()["gamma"] < 0.05
    assert abs(omega - 1.4156) / 1.4156 < 0.01


@pytest.mark.slow
def test_landau_long_rate_and_counts(orc):
    w = workloads.landau_long()
    o = orc.Oracle(w).init()
    d = o.step(w.nsteps)
    t = (np.arange(w.nsteps) + 1) * w.dt
    gamma, omega, peaks = orc.landau_fit(t, d[:, 0], 4.0, 36.0)
    paper = _paper()
    assert abs(-gamma - paper["gamma"]) / paper["gamma"] < 0.02
    assert abs(omega - 1.4156) / 1.4156 < 0.005
    # The paper's oscillation counts: n maxima reached by time t.
    spacing = math.pi / omega
    for rec in paper["oscillation_counts"]:
        assert abs(rec["t"] / spacing - rec["count"]) < 1.0


def test_landau_mass_and_field_history(orc):
    w = workloads.landau_weak()
    o = orc.Oracle(w).init()
    d = o.step(30)
    assert np.all(np.abs(d[:, 1] - d[0, 1]) < 1e-14)        # mass drift
    assert np.all(d[:, 0] > 0) and d[-1, 0] < d[0, 0]        # damping


# ------------------------------------------------------------------ diagnostics

def _wide_landau(alpha=0.01):
    # Weak Landau data on a velocity box wide enough (|v| <= 10, tail of
    # f_M below 1e-22) that the rectangle rule integrates the Gaussian
    # moments to FP64 round-off.
    return workloads.landau_weak().replace(name="landau_wide_64x256", nv=256, vmin=-10.0,
                                           vmax=10.0, amp=(alpha,))


@pytest.mark.parametrize("deltaf", [False, True])
def test_diag_field_closed_form_at_t0(orc, deltaf):
    # f0 = (1 + a cos kx) f_M with k = 2 pi / L: rho = 1 + a cos kx, so
    # E = (a/k) sin kx and (Sections 4.1, 4.3)
    #   ||E||_2 = (dx sum E_i^2)^(1/2) = (a/k) (L/2)^(1/2),
    #   rho_hat_0 = mean rho = 1,   |rho_hat_1| = a/2.
    a, k = 0.01, 0.5
    w = _wide_landau(a)
    o = orc.Oracle(w, deltaf=deltaf).init()
    normE, rho0, rho1 = o.diag_field()
    assert abs(normE - (a / k) * math.sqrt(w.L / 2)) < 1e-14
    assert abs(rho0 - 1.0) < 1e-14
    assert abs(rho1 - a / 2) < 1e-15


@pytest.mark.parametrize("deltaf", [False, True])
@pytest.mark.parametrize("a", [0.01, 0.5])
def test_diag_moments_closed_form_at_t0(orc, deltaf, a):
    # Same f0 (Section 4.2 definitions, f_M = exp(-v^2/2)/sqrt(2 pi)):
    #   L2 = int int f^2 = L (1 + a^2/2) int f_M^2 dv = L (1 + a^2/2) / (2 sqrt(pi)),
    #   energy = 1/2 int int f v^2 + 1/2 int E^2 = L/2 + (a/k)^2 L/4.
    k = 0.5
    w = _wide_landau(a)
    o = orc.Oracle(w, deltaf=deltaf).init()
    l2, energy = o.diag_moments()
    assert abs(l2 - w.L * (1 + a * a / 2) / (2 * math.sqrt(math.pi))) < 1e-13
    assert abs(energy - (w.L / 2 + (a / k) ** 2 * w.L / 4)) < 1e-13


@pytest.mark.parametrize("deltaf", [False, True])
def test_energy_conserved_while_field_energy_moves(orc, deltaf):
    # Vlasov-Poisson conserves the total energy; the split semi-Lagrangian
    # step keeps it up to the O(dt^2) splitting and interpolation errors.
    # Over 50 steps the electric energy swings by ~1e-3 (Landau damping moves
    # it into kinetic energy); the total moves by less than 1% of that swing,
    # so a wrong factor on either term would show.
    w = _wide_landau(0.01)
    o = orc.Oracle(w, deltaf=deltaf).init()
    e0 = o.diag_moments()[1]
    ee0 = 0.5 * o.dx * np.sum(o.E ** 2)
    drift, swing = 0.0, 0.0
    for _ in range(10):
        o.step(5)
        drift = max(drift, abs(o.diag_moments()[1] - e0))
        swing = max(swing, abs(0.5 * o.dx * np.sum(o.E ** 2) - ee0))
    assert swing > 5e-4
    assert drift < 0.01 * swing, (drift, swing)


# ------------------------------------------------------------------ variants

def _trap(w, zero_mean=True):
    return w.replace(poisson="trapezoid", zero_mean=zero_mean)


def test_trapezoid_field_converges_to_fourier(orc):
    # The trapezoidal integral of a smooth periodic rho approaches the exact
    # (Fourier) field at second order in dx (Section 3.2).
    errs = []
    for nx in (32, 64, 128):
        w = workloads.landau_weak().replace(nx=nx, nv=64, degree=17)
        o, ot = orc.Oracle(w), orc.Oracle(_trap(w))
        x = o.x()
        rho = 1.0 + 0.3 * np.cos(0.5 * x) + 0.1 * np.sin(1.5 * x)
        errs.append(np.max(np.abs(ot.poisson(rho) - o.poisson(rho))))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_trapezoid_without_zero_mean(orc):
    # rho - 1 integrated from E_0 = 0: for rho = 1 + a cos(kx) the field is
    # (a/k) sin(kx) up to O(dx^2) and keeps the integration constant; the
    # zero-mean variant is the same field minus its mean.
    w = workloads.landau_weak().replace(nx=128)
    o0, o1 = orc.Oracle(_trap(w, False)), orc.Oracle(_trap(w, True))
    x = o0.x()
    rho = 1.0 + 0.2 * np.cos(0.5 * x)
    E0, E1 = o0.poisson(rho), o1.poisson(rho)
    assert E0[0] == 0.0
    assert np.max(np.abs(E0 - 0.2 / 0.5 * np.sin(0.5 * x))) < 2e-3
    assert np.max(np.abs(E1 - (E0 - E0.mean()))) < 1e-13
    # a wrong background shows up only without the zero-mean step
    E0b, E1b = o0.poisson(rho + 0.01), o1.poisson(rho + 0.01)
    assert np.max(np.abs(E1b - E1)) < 1e-14
    assert np.max(np.abs(E0b - E0)) > 0.05


def test_drive_envelope(orc):
    # a(t0) = 0, a ~ 1 between the ramps, a -> 0 after t_R (Section 4.3).
    o = orc.Oracle(workloads.keen(64, 0.1, 10))
    assert abs(o.drive_amplitude(0.0)) < 1e-15
    assert abs(o.drive_amplitude(188.0) - 1.0) < 1e-4
    # after t_R the bracket vanishes and a -> -eps / (1 - eps), eps ~ 1.0e-3
    eps = 0.5 * (math.tanh(-69.0 / 20.0) - math.tanh(-307.0 / 20.0))
    assert abs(o.drive_amplitude(1000.0) + eps / (1.0 - eps)) < 1e-9
    assert 0.4 < o.drive_amplitude(69.0) < 0.6
    # E_app = emax k a(t) sin(k x - omega t)
    t, x = 150.0, 3.0
    assert abs(o.drive(t, x) - 0.2 * 0.26 * o.drive_amplitude(t) * math.sin(0.26 * x - 0.37 * t)) < 1e-15


def test_drive_enters_the_v_shift(orc):
    # No self-consistent field, delta f = 0 at t = 0 where a(0) = 0: after one
    # step delta f = f_eq(v + dt/2 E_app(dt, x)) - f_eq(v), i.e. the second
    # half step moves the foot by -dt/2 (E - E_app) with E = 0 at t = dt.
    d = workloads.Drive(emax=5.0, tl=0.05, twl=0.01, tr=1e9, twr=1.0, t0=0.0)
    w = workloads.keen(64, 0.1, 1).replace(nv=128, field="zero", drive=d, precision="fp64_deltaf")
    o = orc.Oracle(w).init()
    o.step(1)
    x, v = o.x()[:, None], o.v()[None, :]
    Eapp = np.array([o.drive(w.dt, xi) for xi in o.x()])[:, None]
    fm = lambda vv: np.exp(-vv ** 2 / 2) / math.sqrt(2 * math.pi)
    assert np.max(np.abs(Eapp)) > 0.5
    assert np.max(np.abs(o.f - (fm(v + 0.5 * w.dt * Eapp) - fm(v)))) < 1e-13


def test_rho_modes_normalisation(orc):
    # rho_hat_m = (1/nx) sum rho_i e^{-2 pi i m i/nx}: equals numpy's FFT / nx.
    w = workloads.landau_weak()
    o = orc.Oracle(w)
    rng = np.random.default_rng(2)
    o.rho = rng.standard_normal(w.nx)
    ref = np.abs(np.fft.fft(o.rho))[1:8] / w.nx
    assert np.allclose(o.rho_modes(7), ref, rtol=0, atol=1e-14)


# ----------------------------------------------------------------- B-splines (Section 1.2)

@pytest.mark.parametrize("k", [0, 1, 2, 3, 5, 9, 17])
def test_bspline_basis_matches_library(orc, k):
    # The degree recurrence against scipy's B-spline on the knots 0 .. k+1.
    from scipy.interpolate import BSpline
    be = BSpline.basis_element(np.arange(k + 2.0), extrapolate=False)
    xs = np.linspace(0.013, k + 0.987, 41)
    got = np.array([orc.bspline(k, x) for x in xs])
    assert np.max(np.abs(got - np.nan_to_num(be(xs)))) < 1e-14
    assert orc.bspline(k, -0.5) == 0.0 and orc.bspline(k, k + 1.5) == 0.0


@pytest.mark.parametrize("k", [1, 3, 7, 17])
def test_bspline_partition_of_unity_and_symmetry(orc, k):
    for s in (0.0, 0.21, 0.5, 0.93):
        vals = [orc.bspline(k, s + j) for j in range(k + 1)]
        assert abs(sum(vals) - 1.0) < 1e-14
        assert abs(orc.bspline(k, s + 0.4) - orc.bspline(k, k + 1 - s - 0.4)) < 1e-14


@pytest.mark.parametrize("beta", [0.3, -2.71, 5.5, 13.999])
def test_cubic_spline_advection_matches_library(orc, beta):
    # Periodic cubic spline interpolation evaluated at the feet i + beta.
    from scipy.interpolate import CubicSpline
    n = 32
    u = np.random.default_rng(3).standard_normal(n)
    ref = CubicSpline(np.arange(n + 1.0), np.append(u, u[0]), bc_type="periodic")(
        (np.arange(n) + beta) % n)
    assert np.max(np.abs(orc.advect_line_bspline(u, 3, beta) - ref)) < 1e-13


@pytest.mark.parametrize("k,tol", [(5, 1e-13), (9, 1e-12), (17, 1e-11)])
def test_high_degree_spline_advection_matches_library(orc, k, tol):
    from scipy.interpolate import make_interp_spline
    n = 48
    u = np.random.default_rng(k).standard_normal(n)
    for beta in (0.37, -7.2):
        sp = make_interp_spline(np.arange(n + 1.0), np.append(u, u[0]), k=k, bc_type="periodic")
        ref = sp((np.arange(n) + beta) % n)
        assert np.max(np.abs(orc.advect_line_bspline(u, k, beta) - ref)) < tol


def test_bspline_degree1_is_lagrange1(orc):
    u = np.random.default_rng(5).standard_normal(24)
    for beta in (0.25, -3.6, 11.01):
        assert np.max(np.abs(orc.advect_line_bspline(u, 1, beta) - orc.advect_line(u, 0, beta))) < 1e-15


@pytest.mark.parametrize("k", [3, 17])
@pytest.mark.parametrize("beta", [0, 3, -7])
def test_bspline_integer_shift_is_exact_roll(orc, k, beta):
    # A spline interpolates its data: at an integer shift it returns them.
    u = np.random.default_rng(9).standard_normal(40)
    assert np.max(np.abs(orc.advect_line_bspline(u, k, beta) - np.roll(u, -beta))) < 1e-12


def test_bspline_sweeps_apply_the_line_operator(orc):
    # 2-D sweeps with interp = bspline apply the pinned line operator to every line.
    w = workloads.landau_weak().replace(nx=32, nv=64, interp="bspline", degree=3)
    o = orc.Oracle(w).init()
    f0 = o.f.copy()
    o.advect_x(0.37)
    for j in (0, 17, 63):
        beta = -(w.vmin + j * o.dv) * 0.37 / o.dx
        assert np.max(np.abs(o.f[:, j] - orc.advect_line_bspline(f0[:, j], 3, beta))) < 1e-14
    o.f = f0.copy()
    o.advect_v(0.5)
    for i in (0, 5, 31):
        beta = -o.E[i] * 0.5 / o.dv
        assert np.max(np.abs(o.f[i] - orc.advect_line_bspline(f0[i], 3, beta))) < 1e-14


def test_bspline_landau_rate(orc):
    # Cubic splines resolve weak Landau damping like LAG17 (Section 4.1 rate).
    w = workloads.landau_weak().replace(interp="bspline", degree=3)
    o = orc.Oracle(w).init()
    d = o.step(w.nsteps)
    t = (np.arange(w.nsteps) + 1) * w.dt
    gamma, omega, _ = orc.landau_fit(t, d[:, 0])
    assert abs(-gamma - _paper()["gamma"]) / _paper()["gamma"] < 0.05
    assert abs(omega - 1.4156) / 1.4156 < 0.01


# ------------------------------------------------------- merged v half-steps (Section 1.1)

def test_merged_single_step_is_the_strang_step(orc):
    # With one step there is nothing to merge.
    w = workloads.landau_weak()
    a = orc.Oracle(w).init()
    b = orc.Oracle(w.replace(merge_v=True)).init()
    a.step(1)
    b.step(1)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.E, b.E)


def test_merged_free_streaming_is_unchanged(orc):
    # E = 0: every v-advection is the identity, merged or not.
    w = workloads.free_streaming(32, 32, 8)
    a = orc.Oracle(w).init()
    b = orc.Oracle(w.replace(merge_v=True)).init()
    a.step(8)
    b.step(8)
    assert np.array_equal(a.f, b.f)


def test_merged_differs_at_interpolation_error_level(orc):
    # Two half-shifts vs one full shift differ by the interpolation error:
    # far below the solution scale for LAG17 on smooth data, much larger for LAG3.
    diffs = {}
    for deg in (3, 17):
        w = workloads.landau_weak().replace(degree=deg)
        a = orc.Oracle(w).init()
        b = orc.Oracle(w.replace(merge_v=True)).init()
        a.step(20)
        b.step(20)
        diffs[deg] = np.max(np.abs(a.f - b.f)) / np.max(np.abs(a.f))
    assert 0.0 < diffs[17] < 1e-9
    assert diffs[3] > 10.0 * diffs[17]


def test_merged_landau_rate(orc):
    w = workloads.landau_weak().replace(merge_v=True)
    o = orc.Oracle(w).init()
    d = o.step(w.nsteps)
    t = (np.arange(w.nsteps) + 1) * w.dt
    gamma, omega, _ = orc.landau_fit(t, d[:, 0])
    assert abs(-gamma - _paper()["gamma"]) / _paper()["gamma"] < 0.05
    assert abs(omega - 1.4156) / 1.4156 < 0.01


def test_fp32_rounding_sensitivity_is_far_below_the_gate(orc):
    # The FP32 delta-f gate (1e-5 relative) must sit above what FP32 storage
    # alone causes: rounding delta f0 to FP32 and running 10 strong-Landau steps
    # in FP64 moves delta f by a few FP32 ulps, not more.
    w = workloads.landau_strong()
    a = orc.Oracle(w).init()
    b = orc.Oracle(w).init()
    b.f = b.f.astype(np.float32).astype(np.float64)
    b.update_field()
    a.step(10)
    b.step(10)
    d = np.max(np.abs(a.f - b.f)) / np.max(np.abs(a.f))
    assert 0.0 < d < 1e-6
