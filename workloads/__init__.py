"""Seeded synthetic inputs for the 1D x 1D Vlasov-Poisson workloads.

This module is shared by the CPU oracle, the tests, the benchmark and the
serving harness.  It holds parameters and seeded random draws only: grid
sizes, boxes, time steps, the Gaussian-mixture parameters of the equilibrium
f_eq, the cosine perturbations of the initial condition, and the request
stream of the serving mix.  None of the method's arithmetic lives here; each
side (oracle and HIP library) turns these numbers into f0, weights, symbols
and fields with its own code.

Initial conditions used by every workload have the form

    f0(x, v) = (1 + sum_m amp[m] * cos(kx[m] * x + phase[m])) * f_eq(v)
    f_eq(v)  = sum_g feq_a[g] * exp(-(v - feq_c[g])**2 / (2 * feq_sigma[g]**2))

which covers the Landau (Section 4.1) and bump-on-tail (Section 4.2) initial
data of the paper.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)

PRECISIONS = ("fp64_plain", "fp32_deltaf", "fp64_deltaf", "fp32_plain")


@dataclasses.dataclass(frozen=True)
class Drive:
    """External drive E_app(t, x) = emax k a(t) sin(k x - omega t) of the
    KEEN-wave test (Section 4.3), envelope a(t) from t0, tl, tr, twl, twr."""
    emax: float = 0.2
    k: float = 0.26
    omega: float = 0.37
    t0: float = 0.0
    tl: float = 69.0
    tr: float = 307.0
    twl: float = 20.0
    twr: float = 20.0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    nv: int
    L: float
    vmin: float
    vmax: float
    degree: int
    dt: float
    nsteps: int
    precision: str
    feq_a: Tuple[float, ...]
    feq_c: Tuple[float, ...]
    feq_sigma: Tuple[float, ...]
    amp: Tuple[float, ...]
    kx: Tuple[float, ...]
    phase: Tuple[float, ...]
    field: str = "self_consistent"  # or "zero" (free streaming)
    poisson: str = "fourier"        # or "trapezoid"
    zero_mean: bool = True          # trapezoid only
    drive: Optional[Drive] = None
    interp: str = "lagrange"        # or "bspline" (odd degree k = degree)
    merge_v: bool = False           # merge the v half-steps of consecutive steps
    bitwise_steps: bool = False     # a call of n steps bitwise equal to n single steps

    @property
    def cells(self) -> int:
        return self.nx * self.nv

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


MAXWELLIAN = dict(feq_a=(INV_SQRT_2PI,), feq_c=(0.0,), feq_sigma=(1.0,))


def landau_weak() -> Workload:
    """Weak Landau damping, 64 x 128, plain FP64, 100 steps of dt = 0.1."""
    return Workload("landau_weak_64x128", 64, 128, 4.0 * math.pi, -6.0, 6.0, 17,
                    0.1, 100, "fp64_plain", amp=(0.01,), kx=(0.5,), phase=(0.0,),
                    **MAXWELLIAN)


def landau_strong() -> Workload:
    """Strong Landau damping, 256 x 512, FP32 delta-f, 1000 steps of dt = 0.05."""
    return Workload("landau_strong_256x512", 256, 512, 4.0 * math.pi, -6.0, 6.0, 17,
                    0.05, 1000, "fp32_deltaf", amp=(0.5,), kx=(0.5,), phase=(0.0,),
                    **MAXWELLIAN)


def bump_on_tail() -> Workload:
    """Bump-on-tail, 1024 x 2048, FP32 delta-f about the unperturbed double Maxwellian."""
    return Workload("bump_on_tail_1024x2048", 1024, 2048, 20.0 * math.pi, -9.0, 9.0, 17,
                    0.05, 10000, "fp32_deltaf",
                    feq_a=(0.9 * INV_SQRT_2PI, 0.2 * INV_SQRT_2PI),
                    feq_c=(0.0, 4.5),
                    feq_sigma=(1.0, 1.0 / (2.0 * math.sqrt(2.0))),
                    amp=(0.04,), kx=(0.3,), phase=(0.0,))


def c4_phases(seed: int = 0) -> Tuple[float, ...]:
    rng = np.random.default_rng(seed)
    return tuple(float(p) for p in rng.uniform(0.0, 2.0 * math.pi, 4))


def large_grid() -> Workload:
    """Large-grid throughput case, 4096 x 4096, four seeded-phase modes, 500 steps of dt = 0.02."""
    return Workload("large_grid_4096x4096", 4096, 4096, 4.0 * math.pi, -8.0, 8.0, 17,
                    0.02, 500, "fp32_deltaf",
                    amp=(1e-3,) * 4, kx=tuple(0.5 * m for m in range(1, 5)),
                    phase=c4_phases(0), **MAXWELLIAN)


def keen(n: int = 1024, dt: float = 0.1, nsteps: int = 1000) -> Workload:
    """KEEN waves (Section 4.3): f0 = f_M on [0, 2 pi / k) x [-6, 6), driven by
    E_app with E_max = 0.2, k = 0.26, omega = 0.37, t_L = 69, t_R = 307,
    t_wL = t_wR = 20."""
    d = Drive()
    return Workload(f"keen_{n}x{n}", n, n, 2.0 * math.pi / d.k, -6.0, 6.0, 17, dt, nsteps,
                    "fp32_deltaf", amp=(), kx=(), phase=(), drive=d, **MAXWELLIAN)


def landau_long() -> Workload:
    """Longer weak-Landau run used to pin the damping rate and frequency (t <= 40)."""
    return Workload("landau_long_64x256", 64, 256, 4.0 * math.pi, -8.0, 8.0, 17,
                    0.1, 400, "fp64_plain", amp=(0.01,), kx=(0.5,), phase=(0.0,),
                    **MAXWELLIAN)


def free_streaming(nx: int = 64, nv: int = 64, nsteps: int = 20) -> Workload:
    """Field switched off: f(t, x, v) = f0(x - v t, v)."""
    return Workload(f"free_streaming_{nx}x{nv}", nx, nv, 4.0 * math.pi, -6.0, 6.0, 17,
                    0.1, nsteps, "fp64_plain", amp=(0.05,), kx=(0.5,), phase=(0.3,),
                    field="zero", **MAXWELLIAN)


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    workload: Workload


def serving_mix(n_requests: int = 512, rate: float = 1.0, seed: int = 1,
                steps_range: Tuple[int, int] = (200, 2000),
                nx_pow: Tuple[int, int] = (6, 10), nv_pow: Tuple[int, int] = (7, 11)
                ) -> List[Request]:
    """Serving mix: Poisson arrivals of Landau-type requests of mixed grid sizes.

    nx = 2^U{6..10}, nv = 2^U{7..11}, k ~ U[0.2, 0.6], L = 2 pi / k, amplitude
    log-uniform in [1e-3, 0.5], v in [-8, 8], degree 17, dt = 0.05,
    steps ~ U{200..2000}, FP32 delta-f about the unit Maxwellian.  Arrivals are a
    Poisson process of the given rate (requests per second).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        nx = 2 ** int(rng.integers(nx_pow[0], nx_pow[1] + 1))
        nv = 2 ** int(rng.integers(nv_pow[0], nv_pow[1] + 1))
        k = float(rng.uniform(0.2, 0.6))
        amp = float(math.exp(rng.uniform(math.log(1e-3), math.log(0.5))))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        w = Workload(f"req{r}_{nx}x{nv}", nx, nv, 2.0 * math.pi / k, -8.0, 8.0, 17,
                     0.05, steps, "fp32_deltaf", amp=(amp,), kx=(k,), phase=(0.0,),
                     **MAXWELLIAN)
        out.append(Request(r, float(arrivals[r]), w))
    return out


def all_named() -> List[Workload]:
    return [landau_weak(), landau_strong(), bump_on_tail(), large_grid()]
