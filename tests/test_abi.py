"""CPU-only checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-side configuration logic behaves (no GPU calls)."""
import ctypes
import math
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    with open(os.path.join(ROOT, "include", "vog.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(vog_[A-Za-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def vog():
    from paper_1301_5892_amd import vog as v
    v.load()
    return v


def test_header_declares_the_boundary():
    syms = _header_symbols()
    for name in ["vog_config_validate", "vog_workspace_bytes", "vog_create", "vog_init_perturbed",
                 "vog_set_f", "vog_get_f", "vog_step", "vog_step_batch", "vog_get_E",
                 "vog_get_diag", "vog_sync", "vog_destroy", "vog_strerror"]:
        assert name in syms


def test_library_exports_every_declared_symbol(vog):
    lib = ctypes.CDLL(vog.LIB_PATH)
    missing = [s for s in _header_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(vog.EXPORTS) == set(_header_symbols())


def test_default_config_is_valid(vog):
    c = vog.Config()
    vog.load().vog_config_default(ctypes.byref(c))
    assert vog.load().vog_config_validate(ctypes.byref(c)) == 0
    assert (c.nx, c.nv, c.degree) == (64, 128, 17)


@pytest.mark.parametrize("w", workloads.all_named(), ids=lambda w: w.name)
def test_named_workloads_validate(vog, w):
    c = vog.make_config(w)
    assert vog.load().vog_config_validate(ctypes.byref(c)) == 0
    es = 4 if w.precision == "fp32_deltaf" else 8
    nb = vog.workspace_bytes(c)
    assert nb >= w.nx * w.nv * es
    assert nb < 2 * w.nx * w.nv * es + (4 << 20)


@pytest.mark.parametrize("field,value", [
    ("nx", 12), ("nx", 4), ("nv", 8192), ("nv", 0), ("degree", 4), ("degree", 19),
    ("degree", 0), ("L", 0.0), ("L", float("nan")), ("vmax", -7.0), ("precision", 7),
    ("poisson", 3), ("field", 2), ("n_feq", 0), ("n_feq", 5), ("moments_every", -1),
    ("interp", 2), ("interp", -1), ("merge_v", 2), ("bitwise_steps", 2), ("zero_mean", 3), ("precision", 4),
    ("drive_emax", float("inf"))])
def test_invalid_configs_rejected(vog, field, value):
    c = vog.make_config(workloads.landau_weak())
    setattr(c, field, value)
    assert vog.load().vog_config_validate(ctypes.byref(c)) == vog.EINVAL
    assert vog.workspace_bytes(c) == 0
    assert len(vog.load().vog_last_error()) > 0


@pytest.mark.parametrize("precision", ["fp32_plain", "fp64_deltaf"])
@pytest.mark.parametrize("interp", ["lagrange", "bspline"])
def test_variant_configs_validate(vog, precision, interp):
    w = workloads.landau_strong().replace(precision=precision, interp=interp, merge_v=True)
    c = vog.make_config(w)
    assert vog.load().vog_config_validate(ctypes.byref(c)) == 0
    es = 4 if precision == "fp32_plain" else 8
    nb = vog.workspace_bytes(c)
    assert nb >= w.nx * w.nv * es
    # B-splines add one table of 1/D_m per line length
    base = vog.workspace_bytes(vog.make_config(w.replace(interp="lagrange")))
    assert (nb > base) == (interp == "bspline")


def test_drive_widths_must_be_positive(vog):
    c = vog.make_config(workloads.keen(64))
    assert vog.load().vog_config_validate(ctypes.byref(c)) == 0
    c.drive_twl = 0.0
    assert vog.load().vog_config_validate(ctypes.byref(c)) == vog.EINVAL


def test_degree_must_fit_the_grid(vog):
    c = vog.make_config(workloads.landau_weak().replace(nx=16))
    assert vog.load().vog_config_validate(ctypes.byref(c)) == vog.EINVAL
    c.degree = 15
    assert vog.load().vog_config_validate(ctypes.byref(c)) == 0


def test_feq_sigma_must_be_positive(vog):
    c = vog.make_config(workloads.landau_weak())
    c.feq_sigma[0] = 0.0
    assert vog.load().vog_config_validate(ctypes.byref(c)) == vog.EINVAL


def test_null_arguments_fail_cleanly(vog):
    L = vog.load()
    assert L.vog_config_validate(None) == vog.EINVAL
    out = ctypes.c_void_p()
    assert L.vog_create(None, None, 0, None, ctypes.byref(out)) == vog.EINVAL
    assert L.vog_step(None, 0.1, 1) == vog.EINVAL
    assert L.vog_sync(None) == vog.EINVAL
    st = (ctypes.c_int * 1)()
    assert L.vog_sync_batch(None, 1, st) == vog.EINVAL
    assert L.vog_sync_batch((vog._P * 1)(None), 1, st) == vog.EINVAL
    assert L.vog_sync_batch((vog._P * 1)(None), 0, st) == vog.EINVAL
    L.vog_destroy(None)
    assert L.vog_strerror(vog.ENONFINITE) == b"non-finite field"


def test_serving_mix_is_seeded():
    a = workloads.serving_mix(64, rate=2.0)
    b = workloads.serving_mix(64, rate=2.0)
    assert [(r.arrival, r.workload) for r in a] == [(r.arrival, r.workload) for r in b]
    for r in a:
        assert 64 <= r.workload.nx <= 1024 and 128 <= r.workload.nv <= 2048
        assert 200 <= r.workload.nsteps <= 2000
        assert 1e-3 <= r.workload.amp[0] <= 0.5
        assert abs(r.workload.L * r.workload.kx[0] - 2 * math.pi) < 1e-12


def test_noalloc_sync_batch_rejects_bad_arguments_on_the_host(vog):
    # argument checks come before any device work
    L = vog.load()
    st = (ctypes.c_int * 2)()
    assert L.vog_sync_batch_noalloc(None, 1, st) == vog.EINVAL
    assert L.vog_sync_batch_noalloc((vog._P * 1)(None), 1, st) == vog.EINVAL
    assert L.vog_sync_batch_noalloc((vog._P * 1)(None), 0, st) == vog.EINVAL
    n = vog.NOALLOC_MAX_SIMS + 1
    assert L.vog_sync_batch_noalloc((vog._P * n)(), n, (ctypes.c_int * n)()) == vog.EINVAL
