"""The C-ABI library loads and exports every entry point declared in
include/libtdse.h; argument validation runs on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2507_04115_amd import binding as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    """A clean checkout has no libtdse.so: build it (hipcc cross-compiles for
    gfx950 without a GPU), or skip the module when no HIP compiler is here."""
    if os.path.exists(L.LIB_PATH):
        return
    from paper_2507_04115_amd import build as hip_build

    if not os.path.exists(hip_build.HIPCC):
        pytest.skip(f"libtdse.so is not built and {hip_build.HIPCC} is missing",
                    allow_module_level=True)
    hip_build.build()


_ensure_built()


def _declared():
    txt = open(os.path.join(ROOT, "include", "libtdse.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tdse_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = L.load()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.exported_names())


def test_version_and_status_strings():
    assert "gfx950" in L.tdse_version()
    lib = L.load()
    for st in range(0, -7, -1):
        assert lib.tdse_status_string(st)
    assert lib.tdse_status_string(-99) == b"unknown status"


def _create(p, ns, out=True):
    lib = L.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int32 * len(ns))(*ns)
    return lib.tdse_plan_create(ctypes.byref(p), len(ns), arr, 0, 0,
                                ctypes.byref(h) if out else None)


@pytest.mark.parametrize("field,value,msg", [
    ("dx", 0.0, "dx"), ("dt", -1.0, "dt"), ("a", -1.0, "soft-core"),
    ("mask_fraction", 1.5, "mask_fraction"), ("mask_fraction", 0.5, "mask_fraction"),
    ("nt", -3, "nt"), ("flags", 1, "flags"),
])
def test_plan_create_rejects_bad_params_before_touching_the_device(field, value, msg):
    p = L.make_params(0.2, 0.05, 1.2, 100)
    setattr(p, field, value)
    assert _create(p, [256]) == L.TDSE_E_INVALID
    assert msg in L.load().tdse_last_error().decode()


def test_plan_create_rejects_bad_sizes():
    p = L.make_params(0.2, 0.05, 1.2, 100)
    assert _create(p, [8]) == L.TDSE_E_INVALID
    assert _create(p, [20000]) == L.TDSE_E_UNSUPPORTED
    assert _create(p, [256], out=False) == L.TDSE_E_INVALID


def test_yield_and_propagate_validation():
    lib = L.load()
    assert lib.tdse_harmonic_yield(0, 100, 0.05, 0.057, 21, 31, 16, None, 16, 16, None, None) == L.TDSE_E_INVALID
    assert lib.tdse_harmonic_yield(1, 100, 0.05, 0.057, 31, 21, 16, None, 16, 16, None, None) == L.TDSE_E_INVALID
    assert lib.tdse_harmonic_yield(1, 100, 0.05, 0.057, 21, 31, 8, None, 16, 16, None, None) == L.TDSE_E_INVALID
    assert "aligned" in lib.tdse_last_error().decode()
    assert lib.tdse_propagate_batch(None, 16, None, 16, None, None, None, None, None) == L.TDSE_E_INVALID
    assert lib.tdse_adjoint_batch(None, 16, None, 16, 16, None, None, None) == L.TDSE_E_INVALID


def test_harmonic_band_matches_definition():
    k_lo, nk = L.tdse_harmonic_band(22047, 0.05, 0.057, 21, 31)
    import numpy as np
    dw = 2 * np.pi / (22048 * 0.05)
    k = np.arange(22048 // 2 + 1)
    sel = k[(k * dw >= 21 * 0.057) & (k * dw <= 31 * 0.057)]
    assert (k_lo, nk) == (sel[0], len(sel))


def test_resample_validation_before_any_launch():
    """tdse_resample_field refuses bad sizes on the host (no device needed):
    a padded length M dt_coarse / dt that is not an integer or is below
    max(M, nt+1), a short workspace, an empty batch, misalignment."""
    lib = L.load()
    f = lib.tdse_resample_field
    bad = [
        (4, 64, 0.3, 0.07, 100, 16, 16, 16 * 4 * 33, 16, None),    # 64 * 0.3 / 0.07 not an integer
        (4, 64, 0.3, 0.1, 192, 16, 16, 16 * 4 * 33, 16, None),     # M' = 192 < nt + 1
        (4, 64, 0.3, 0.1, 100, 16, 16, 16 * 4 * 33 - 1, 16, None), # work too small
        (0, 64, 0.3, 0.1, 100, 16, 16, 16 * 4 * 33, 16, None),     # empty batch
        (4, 1, 0.3, 0.1, 100, 16, 16, 16 * 4 * 33, 16, None),      # one sample
        (4, 64, 0.3, 0.1, 100, 16, 24, 16 * 4 * 33, 16, None),     # work not 16-byte aligned
        (4, 64, 0.3, 0.1, 100, None, 16, 16 * 4 * 33, 16, None),   # no input
    ]
    for args in bad:
        assert f(*args) == L.TDSE_E_INVALID, args
        assert lib.tdse_last_error().decode()


def test_energy_integral_validation_before_any_launch():
    """tdse_energy_integral refuses an empty batch, a grid of one point, a
    NaN or +inf threshold and NULL arrays on the host."""
    lib = L.load()
    f = lib.tdse_energy_integral
    assert f(0, 8, 16, 16, 0.0, 16, None) == L.TDSE_E_INVALID
    assert f(2, 1, 16, 16, 0.0, 16, None) == L.TDSE_E_INVALID
    assert f(2, 8, 16, 16, float("nan"), 16, None) == L.TDSE_E_INVALID
    assert f(2, 8, 16, 16, float("inf"), 16, None) == L.TDSE_E_INVALID
    assert f(2, 8, None, 16, 0.0, 16, None) == L.TDSE_E_INVALID
    assert "required" in lib.tdse_last_error().decode()
