"""ctypes binding of libvog (include/vog.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libvog.so.  PyTorch is
used for device memory (the workspace tensor handed to vog_create) and for
streams.  If libvog.so has not been built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvog.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EBUSY = 0, -1, -2, -3, -4, -5
NOALLOC_MAX_SIMS = 1024  # VOG_NOALLOC_MAX_SIMS of vog.h
FP64_PLAIN, FP32_DELTAF, FP64_DELTAF, FP32_PLAIN = 0, 1, 2, 3
INTERP_LAGRANGE, INTERP_BSPLINE = 0, 1
POISSON_FOURIER, POISSON_TRAPEZOID = 0, 1
FIELD_SELF_CONSISTENT, FIELD_ZERO = 0, 1
MAX_FEQ = 4
NUM_KINDS = 8
KIND_NAMES = ("sweep_v", "sweep_x", "transpose_vx", "transpose_xv_rho", "field", "moments",
              "rho_reduce", "sweep_vv")
PRECISION = {"fp64_plain": FP64_PLAIN, "fp32_deltaf": FP32_DELTAF, "fp64_deltaf": FP64_DELTAF,
             "fp32_plain": FP32_PLAIN}
INTERP = {"lagrange": INTERP_LAGRANGE, "bspline": INTERP_BSPLINE}


class VogError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nv", ctypes.c_int),
                ("L", ctypes.c_double), ("vmin", ctypes.c_double), ("vmax", ctypes.c_double),
                ("degree", ctypes.c_int), ("precision", ctypes.c_int),
                ("poisson", ctypes.c_int), ("field", ctypes.c_int),
                ("n_feq", ctypes.c_int),
                ("feq_a", ctypes.c_double * MAX_FEQ), ("feq_c", ctypes.c_double * MAX_FEQ),
                ("feq_sigma", ctypes.c_double * MAX_FEQ),
                ("moments_every", ctypes.c_int), ("zero_mean", ctypes.c_int),
                ("drive_emax", ctypes.c_double), ("drive_k", ctypes.c_double),
                ("drive_omega", ctypes.c_double), ("drive_t0", ctypes.c_double),
                ("drive_tl", ctypes.c_double), ("drive_tr", ctypes.c_double),
                ("drive_twl", ctypes.c_double), ("drive_twr", ctypes.c_double),
                ("interp", ctypes.c_int), ("merge_v", ctypes.c_int),
                ("bitwise_steps", ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("normE", ctypes.c_double),
                ("rho0", ctypes.c_double), ("abs_rho1", ctypes.c_double),
                ("l2", ctypes.c_double), ("energy", ctypes.c_double),
                ("finite", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("abs_rho_modes", ctypes.c_double * 7)]


DIAG_DTYPE = np.dtype([("step", np.int64), ("t", np.float64), ("normE", np.float64),
                       ("rho0", np.float64), ("abs_rho1", np.float64), ("l2", np.float64),
                       ("energy", np.float64), ("finite", np.int32), ("reserved", np.int32),
                       ("abs_rho_modes", np.float64, (7,))])
assert DIAG_DTYPE.itemsize == ctypes.sizeof(Diag)

EXPORTS = ["vog_config_default", "vog_config_validate", "vog_workspace_bytes", "vog_create",
           "vog_init_perturbed", "vog_set_f", "vog_get_f", "vog_get_raw", "vog_get_E",
           "vog_set_E", "vog_step", "vog_step_batch", "vog_sweep", "vog_get_diag",
           "vog_state_bytes", "vog_get_state", "vog_set_state", "vog_get_time", "vog_sync", "vog_sync_batch",
           "vog_sync_batch_noalloc", "vog_destroy", "vog_strerror", "vog_last_error", "vog_profile_enable",
           "vog_profile_read", "vog_build_info"]

_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def load() -> ctypes.CDLL:
    """Loads libvog.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python -m paper_1301_5892_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    cp = ctypes.POINTER(Config)
    sig = {
        "vog_config_default": (None, [cp]),
        "vog_config_validate": (ctypes.c_int, [cp]),
        "vog_workspace_bytes": (ctypes.c_size_t, [cp]),
        "vog_create": (ctypes.c_int, [cp, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
        "vog_init_perturbed": (ctypes.c_int, [_P, ctypes.c_int, _D, _D, _D]),
        "vog_set_f": (ctypes.c_int, [_P, _D]),
        "vog_get_f": (ctypes.c_int, [_P, _D]),
        "vog_get_raw": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int)]),
        "vog_get_E": (ctypes.c_int, [_P, _D]),
        "vog_set_E": (ctypes.c_int, [_P, _D]),
        "vog_step": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int]),
        "vog_step_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _D, ctypes.c_int]),
        "vog_sweep": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double]),
        "vog_get_diag": (ctypes.c_int, [_P, ctypes.POINTER(Diag), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
        "vog_state_bytes": (ctypes.c_size_t, [_P]),
        "vog_get_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
        "vog_set_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
        "vog_get_time": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]),
        "vog_sync": (ctypes.c_int, [_P]),
        "vog_sync_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "vog_sync_batch_noalloc": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "vog_destroy": (None, [_P]),
        "vog_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "vog_last_error": (ctypes.c_char_p, []),
        "vog_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
        "vog_profile_read": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
        "vog_build_info": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int, where: str) -> None:
    if rc != OK:
        L = load()
        raise VogError(rc, where, f"{L.vog_strerror(rc).decode()}: {L.vog_last_error().decode()}")


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def make_config(w, moments_every: int = 0, precision: Optional[str] = None) -> Config:
    """vog_config of a workloads.Workload."""
    c = Config()
    load().vog_config_default(ctypes.byref(c))
    c.nx, c.nv = w.nx, w.nv
    c.L, c.vmin, c.vmax = w.L, w.vmin, w.vmax
    c.degree = w.degree
    c.precision = PRECISION[precision or w.precision]
    c.poisson = POISSON_TRAPEZOID if w.poisson == "trapezoid" else POISSON_FOURIER
    c.zero_mean = int(bool(w.zero_mean))
    c.field = FIELD_ZERO if w.field == "zero" else FIELD_SELF_CONSISTENT
    if w.drive is not None:
        d = w.drive
        c.drive_emax, c.drive_k, c.drive_omega = d.emax, d.k, d.omega
        c.drive_t0, c.drive_tl, c.drive_tr = d.t0, d.tl, d.tr
        c.drive_twl, c.drive_twr = d.twl, d.twr
    c.n_feq = len(w.feq_a)
    for g in range(c.n_feq):
        c.feq_a[g], c.feq_c[g], c.feq_sigma[g] = w.feq_a[g], w.feq_c[g], w.feq_sigma[g]
    c.moments_every = moments_every
    c.interp = INTERP[w.interp]
    c.merge_v = int(bool(w.merge_v))
    c.bitwise_steps = int(bool(w.bitwise_steps))
    return c


def workspace_bytes(cfg: Config) -> int:
    return int(load().vog_workspace_bytes(ctypes.byref(cfg)))


def current_stream_handle(device=None) -> int:
    import torch
    return int(torch.cuda.current_stream(device).cuda_stream)


class Sim:
    """One simulation: f (or delta f) and E resident in a torch-allocated
    device workspace, all work enqueued on one HIP stream."""

    def __init__(self, w, moments_every: int = 0, precision: Optional[str] = None,
                 stream=None, workspace=None):
        import torch
        L = load()
        self.w = w
        self.cfg = make_config(w, moments_every, precision)
        _check(L.vog_config_validate(ctypes.byref(self.cfg)), "vog_config_validate")
        self.nbytes = workspace_bytes(self.cfg)
        if workspace is None:
            workspace = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        self.workspace = workspace  # kept alive for the sim's lifetime
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _P()
        _check(L.vog_create(ctypes.byref(self.cfg), ctypes.c_void_p(workspace.data_ptr()),
                            self.nbytes, ctypes.c_void_p(int(self.stream.cuda_stream)),
                            ctypes.byref(h)), "vog_create")
        self.handle = h
        self.nx, self.nv = w.nx, w.nv

    # -- lifetime
    def close(self) -> None:
        if self.handle:
            load().vog_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state
    def init(self, amp=None, kx=None, phase=None) -> "Sim":
        w = self.w
        amp = np.ascontiguousarray(w.amp if amp is None else amp, dtype=np.float64)
        kx = np.ascontiguousarray(w.kx if kx is None else kx, dtype=np.float64)
        phase = np.ascontiguousarray(w.phase if phase is None else phase, dtype=np.float64)
        _check(load().vog_init_perturbed(self.handle, amp.size, _dp(amp), _dp(kx), _dp(phase)),
               "vog_init_perturbed")
        return self

    def set_f(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.nx, self.nv)
        _check(load().vog_set_f(self.handle, _dp(f)), "vog_set_f")

    def get_f(self) -> np.ndarray:
        out = np.zeros((self.nx, self.nv))
        _check(load().vog_get_f(self.handle, _dp(out)), "vog_get_f")
        return out

    def get_raw(self) -> np.ndarray:
        es = 4 if self.cfg.precision in (FP32_DELTAF, FP32_PLAIN) else 8
        out = np.zeros((self.nx, self.nv), dtype=np.float32 if es == 4 else np.float64)
        eb = ctypes.c_int()
        _check(load().vog_get_raw(self.handle, out.ctypes.data_as(_P), out.nbytes,
                                  ctypes.byref(eb)), "vog_get_raw")
        return out

    def get_E(self) -> np.ndarray:
        out = np.zeros(self.nx)
        _check(load().vog_get_E(self.handle, _dp(out)), "vog_get_E")
        return out

    def set_E(self, E: np.ndarray) -> None:
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.nx
        _check(load().vog_set_E(self.handle, _dp(E)), "vog_set_E")

    # -- time stepping
    def step(self, nsteps: int = 1, dt: Optional[float] = None) -> None:
        dt = self.w.dt if dt is None else dt
        _check(load().vog_step(self.handle, float(dt), int(nsteps)), "vog_step")

    def advect_v(self, tau: float) -> None:
        _check(load().vog_sweep(self.handle, 0, float(tau)), "vog_sweep(v)")

    def advect_x(self, dt: float) -> None:
        _check(load().vog_sweep(self.handle, 1, float(dt)), "vog_sweep(x)")

    def update_field(self) -> None:
        _check(load().vog_sweep(self.handle, 2, 0.0), "vog_sweep(field)")

    def sync(self) -> None:
        _check(load().vog_sync(self.handle), "vog_sync")

    def time(self):
        st = ctypes.c_int64()
        t = ctypes.c_double()
        _check(load().vog_get_time(self.handle, ctypes.byref(st), ctypes.byref(t)), "vog_get_time")
        return st.value, t.value

    # -- diagnostics
    def diag(self, cap: int = 4096) -> np.ndarray:
        buf = (Diag * cap)()
        n = ctypes.c_int()
        _check(load().vog_get_diag(self.handle, buf, cap, ctypes.byref(n)), "vog_get_diag")
        arr = np.frombuffer(bytes(buf), dtype=DIAG_DTYPE, count=cap)
        return arr[: n.value].copy()

    # -- checkpoint
    def get_state(self) -> bytes:
        L = load()
        nb = int(L.vog_state_bytes(self.handle))
        buf = ctypes.create_string_buffer(nb)
        _check(L.vog_get_state(self.handle, ctypes.cast(buf, _P), nb), "vog_get_state")
        return buf.raw

    def set_state(self, state: bytes) -> None:
        buf = ctypes.create_string_buffer(state, len(state))
        _check(load().vog_set_state(self.handle, ctypes.cast(buf, _P), len(state)), "vog_set_state")

    # -- profiling
    def profile(self, on: bool) -> None:
        _check(load().vog_profile_enable(self.handle, int(on)), "vog_profile_enable")

    def profile_read(self):
        ms = np.zeros(NUM_KINDS)
        n = (ctypes.c_int64 * NUM_KINDS)()
        _check(load().vog_profile_read(self.handle, _dp(ms), n, NUM_KINDS), "vog_profile_read")
        return {KIND_NAMES[k]: (float(ms[k]), int(n[k])) for k in range(NUM_KINDS)}


def step_batch(sims: Sequence[Sim], nsteps: int, dts: Optional[Sequence[float]] = None) -> None:
    """Grouped launches over several sims that share one stream."""
    n = len(sims)
    arr = (_P * n)(*[s.handle for s in sims])
    dt = np.ascontiguousarray([s.w.dt for s in sims] if dts is None else dts, dtype=np.float64)
    _check(load().vog_step_batch(arr, n, _dp(dt), int(nsteps)), "vog_step_batch")


def sync_batch(sims: Sequence[Sim]) -> List[bool]:
    """Waits for the shared stream once; whether each sim's last recorded
    field is finite."""
    n = len(sims)
    arr = (_P * n)(*[s.handle for s in sims])
    st = (ctypes.c_int * n)()
    _check(load().vog_sync_batch(arr, n, st), "vog_sync_batch")
    return [st[k] == OK for k in range(n)]


def build_info() -> str:
    return load().vog_build_info().decode()
