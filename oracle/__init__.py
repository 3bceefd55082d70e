"""CPU FP64 oracle for the 1D x 1D Vlasov-Poisson split step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (`paper_1301_5892_amd`), and neither imports the other; both
take their inputs from `workloads`.

The arithmetic lives in `vp_oracle.c` (plain C, FP64, direct circulant
stencil, direct-DFT Poisson solve; see that file for the paper passages each
function follows).  This module builds it with gcc, loads it with ctypes and
adds the Landau-damping fit used to read the damping rate and frequency off
an ||E||_2 history (Section 4.1).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_FEQ = 4


def build(force: bool = True) -> str:
    """Compile vp_oracle.c into liboracle.so (gcc, -O2, OpenMP over lines)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nv", ctypes.c_int),
                ("L", ctypes.c_double), ("vmin", ctypes.c_double), ("vmax", ctypes.c_double),
                ("degree", ctypes.c_int), ("deltaf", ctypes.c_int), ("field_zero", ctypes.c_int),
                ("n_feq", ctypes.c_int),
                ("feq_a", ctypes.c_double * MAX_FEQ), ("feq_c", ctypes.c_double * MAX_FEQ),
                ("feq_sigma", ctypes.c_double * MAX_FEQ),
                ("poisson", ctypes.c_int), ("zero_mean", ctypes.c_int),
                ("drive_emax", ctypes.c_double), ("drive_k", ctypes.c_double),
                ("drive_omega", ctypes.c_double), ("drive_t0", ctypes.c_double),
                ("drive_tl", ctypes.c_double), ("drive_tr", ctypes.c_double),
                ("drive_twl", ctypes.c_double), ("drive_twr", ctypes.c_double),
                ("interp", ctypes.c_int), ("merge_v", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        cp = ctypes.POINTER(_Cfg)
        L.orc_lagrange_weights.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.orc_split_shift.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_long), _D]
        L.orc_circulant_row.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D]
        L.orc_advect_line.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_bspline.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_bspline.restype = ctypes.c_double
        L.orc_advect_line_bspline.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, _D]
        L.orc_feq.argtypes = [cp, ctypes.c_double]
        L.orc_feq.restype = ctypes.c_double
        L.orc_init.argtypes = [cp, ctypes.c_int, _D, _D, _D, _D]
        L.orc_advect_x.argtypes = [cp, ctypes.c_double, _D, _D]
        L.orc_advect_v.argtypes = [cp, _D, ctypes.c_double, _D, _D]
        L.orc_rho.argtypes = [cp, _D, _D]
        L.orc_poisson.argtypes = [cp, _D, _D]
        L.orc_solve.argtypes = [cp, _D, _D]
        L.orc_field.argtypes = [cp, _D, _D, _D]
        L.orc_step.argtypes = [cp, ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.orc_run.argtypes = [cp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_drive_amplitude.argtypes = [cp, ctypes.c_double]
        L.orc_drive_amplitude.restype = ctypes.c_double
        L.orc_drive.argtypes = [cp, ctypes.c_double, ctypes.c_double]
        L.orc_drive.restype = ctypes.c_double
        L.orc_rho_modes.argtypes = [cp, _D, ctypes.c_int, _D]
        L.orc_diag_field.argtypes = [cp, _D, _D, _D]
        L.orc_diag_moments.argtypes = [cp, _D, _D, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------- 1D pieces

def lagrange_weights(d: int, s: float) -> np.ndarray:
    """w[j + d], j = -d .. d+1: Lagrange 2d+1 coefficients (Section 1.2)."""
    w = np.zeros(2 * d + 2)
    lib().orc_lagrange_weights(int(d), float(s), _p(w))
    return w


def split_shift(beta: float) -> Tuple[int, float]:
    b = ctypes.c_long()
    s = ctypes.c_double()
    lib().orc_split_shift(float(beta), ctypes.byref(b), ctypes.byref(s))
    return b.value, s.value


def circulant_row(n: int, d: int, beta: float) -> np.ndarray:
    """(a_0 .. a_{n-1}) of A = C(a_0 .. a_{n-1}) (Section 1.2)."""
    a = np.zeros(n)
    lib().orc_circulant_row(int(n), int(d), float(beta), _p(a))
    return a


def advect_line(u: np.ndarray, d: int, beta: float) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().orc_advect_line(u.size, int(d), float(beta), _p(u), _p(out))
    return out


def bspline(k: int, x: float) -> float:
    """B^k_0(x) on the unit mesh (Section 1.2 recurrence)."""
    return lib().orc_bspline(int(k), float(x))


def advect_line_bspline(u: np.ndarray, k: int, beta: float) -> np.ndarray:
    """Periodic B-spline interpolation of degree k of u at the feet i + beta."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().orc_advect_line_bspline(u.size, int(k), float(beta), _p(u), _p(out))
    return out


# ---------------------------------------------------------------- 2D model

class Oracle:
    """Oracle state for one workload: f (or delta f) and E, both FP64."""

    def __init__(self, w, deltaf: Optional[bool] = None):
        if deltaf is None:
            deltaf = w.precision.endswith("deltaf")
        self.w = w
        c = _Cfg()
        c.nx, c.nv = w.nx, w.nv
        c.L, c.vmin, c.vmax = w.L, w.vmin, w.vmax
        c.degree = w.degree
        c.deltaf = int(bool(deltaf))
        c.field_zero = int(w.field == "zero")
        c.n_feq = len(w.feq_a)
        for g in range(c.n_feq):
            c.feq_a[g], c.feq_c[g], c.feq_sigma[g] = w.feq_a[g], w.feq_c[g], w.feq_sigma[g]
        c.poisson = 1 if w.poisson == "trapezoid" else 0
        c.zero_mean = int(bool(w.zero_mean))
        c.interp = 1 if w.interp == "bspline" else 0
        c.merge_v = int(bool(w.merge_v))
        if w.drive is not None:
            d = w.drive
            c.drive_emax, c.drive_k, c.drive_omega = d.emax, d.k, d.omega
            c.drive_t0, c.drive_tl, c.drive_tr = d.t0, d.tl, d.tr
            c.drive_twl, c.drive_twr = d.twl, d.twr
        self.cfg = c
        self.deltaf = bool(deltaf)
        self.f = np.zeros((w.nx, w.nv))
        self.E = np.zeros(w.nx)
        self.rho = np.zeros(w.nx)
        self.step_count = 0
        self.t = 0.0

    @property
    def dx(self) -> float:
        return self.w.L / self.w.nx

    @property
    def dv(self) -> float:
        return (self.w.vmax - self.w.vmin) / self.w.nv

    def x(self) -> np.ndarray:
        return np.arange(self.w.nx) * self.dx

    def v(self) -> np.ndarray:
        return self.w.vmin + np.arange(self.w.nv) * self.dv

    def feq(self, v: float) -> float:
        return lib().orc_feq(ctypes.byref(self.cfg), float(v))

    def feq_grid(self) -> np.ndarray:
        return np.array([self.feq(v) for v in self.v()])

    def init(self, amp=None, kx=None, phase=None) -> "Oracle":
        w = self.w
        amp = np.ascontiguousarray(w.amp if amp is None else amp, dtype=np.float64)
        kx = np.ascontiguousarray(w.kx if kx is None else kx, dtype=np.float64)
        phase = np.ascontiguousarray(w.phase if phase is None else phase, dtype=np.float64)
        lib().orc_init(ctypes.byref(self.cfg), amp.size, _p(amp), _p(kx), _p(phase), _p(self.f))
        self.update_field()
        self.step_count = 0
        self.t = 0.0
        return self

    def set_full_f(self, f_full: np.ndarray) -> None:
        f_full = np.asarray(f_full, dtype=np.float64).reshape(self.w.nx, self.w.nv)
        self.f = np.ascontiguousarray(f_full - self.feq_grid()[None, :] if self.deltaf else f_full)
        self.update_field()

    def full_f(self) -> np.ndarray:
        return self.f + self.feq_grid()[None, :] if self.deltaf else self.f.copy()

    def update_field(self) -> None:
        lib().orc_field(ctypes.byref(self.cfg), _p(self.f), _p(self.E), _p(self.rho))

    # single sweeps (exposed for sweep-level parity tests)
    def advect_x(self, dt: float) -> None:
        out = np.empty_like(self.f)
        lib().orc_advect_x(ctypes.byref(self.cfg), float(dt), _p(self.f), _p(out))
        self.f = out

    def advect_v(self, tau: float, E: Optional[np.ndarray] = None) -> None:
        E = self.E if E is None else np.ascontiguousarray(E, dtype=np.float64)
        out = np.empty_like(self.f)
        lib().orc_advect_v(ctypes.byref(self.cfg), _p(E), float(tau), _p(self.f), _p(out))
        self.f = out

    def rho_of(self) -> np.ndarray:
        rho = np.zeros(self.w.nx)
        lib().orc_rho(ctypes.byref(self.cfg), _p(self.f), _p(rho))
        return rho

    def poisson(self, rho: np.ndarray) -> np.ndarray:
        """E from rho with the workload's field solve (Fourier or trapezoid)."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        E = np.zeros(self.w.nx)
        lib().orc_solve(ctypes.byref(self.cfg), _p(rho), _p(E))
        return E

    def step(self, nsteps: int = 1, dt: Optional[float] = None) -> np.ndarray:
        """Advance nsteps Strang steps; returns (nsteps, 3) records of
        ||E||_2, rho_hat_0, |rho_hat_1| after each step."""
        dt = self.w.dt if dt is None else dt
        diag = np.zeros((nsteps, 3))
        lib().orc_run(ctypes.byref(self.cfg), float(self.t), float(dt), int(nsteps), _p(self.f),
                      _p(self.E), _p(diag))
        self.step_count += nsteps
        self.t += nsteps * dt
        if nsteps:
            self.rho = self.rho_of()
        return diag

    def diag_field(self) -> np.ndarray:
        out = np.zeros(3)
        lib().orc_diag_field(ctypes.byref(self.cfg), _p(self.rho), _p(self.E), _p(out))
        return out

    def rho_modes(self, nmodes: int = 7) -> np.ndarray:
        out = np.zeros(nmodes)
        lib().orc_rho_modes(ctypes.byref(self.cfg), _p(self.rho), int(nmodes), _p(out))
        return out

    def drive_amplitude(self, t: float) -> float:
        return lib().orc_drive_amplitude(ctypes.byref(self.cfg), float(t))

    def drive(self, t: float, x: float) -> float:
        return lib().orc_drive(ctypes.byref(self.cfg), float(t), float(x))

    def diag_moments(self) -> np.ndarray:
        out = np.zeros(2)
        lib().orc_diag_moments(ctypes.byref(self.cfg), _p(self.f), _p(self.E), _p(out))
        return out


# ---------------------------------------------------------------- Landau fit

def landau_fit(t: np.ndarray, normE: np.ndarray, tmin: float = 0.0,
               tmax: float = math.inf) -> Tuple[float, float, np.ndarray]:
    """Damping rate and frequency from an ||E||_2 history (Section 4.1).

    Local maxima of ln ||E||_2 inside [tmin, tmax] are refined by a parabola
    through the three samples around each maximum; a least-squares line through
    the refined maxima gives the rate gamma (slope of ln ||E||_2, negative when
    damped); ||E||_2 peaks twice per period, so omega = pi / mean spacing.
    Returns (gamma, omega, peak_times).
    """
    t = np.asarray(t, dtype=np.float64)
    y = np.log(np.asarray(normE, dtype=np.float64))
    pt, py = [], []
    for k in range(1, len(y) - 1):
        if y[k] > y[k - 1] and y[k] >= y[k + 1] and tmin <= t[k] <= tmax:
            h = t[k + 1] - t[k]
            den = y[k - 1] - 2.0 * y[k] + y[k + 1]
            off = 0.5 * (y[k - 1] - y[k + 1]) / den if den != 0.0 else 0.0
            pt.append(t[k] + off * h)
            py.append(y[k] - 0.25 * (y[k - 1] - y[k + 1]) * off)
    pt, py = np.array(pt), np.array(py)
    if len(pt) < 3:
        return float("nan"), float("nan"), pt
    gamma = float(np.polyfit(pt, py, 1)[0])
    omega = float(math.pi / np.mean(np.diff(pt)))
    return gamma, omega, pt
