"""Pins of the seeded input generators against the workload definitions
(tests/golden/workload_constants.json)."""
import json
import math
import os

import numpy as np

import tdse_inputs as ti

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "workload_constants.json")))


def test_unit_conversions():
    assert abs(ti.field_amplitude(1.5e14) - G["e0_at_1p5e14_wcm2_au"]["value"]) < G["e0_at_1p5e14_wcm2_au"]["tol"]
    assert abs(ti.omega_from_wavelength(800) - G["omega_800nm_au"]["value"]) < G["omega_800nm_au"]["tol"]
    assert abs(ti.omega_from_wavelength(1300) - G["omega_1300nm_au"]["value"]) < G["omega_1300nm_au"]["tol"]
    assert ti.IP_ARGON == G["ip_argon_au"]["value"]


def test_step_counts():
    assert ti.cfg1_single().nt == G["nt_single"]["value"]
    assert ti.cfg2_focus().nt == G["nt_focus"]["value"]
    assert ti.cfg5_volume(2, 2).nt == G["nt_volume"]["value"]


def test_gaussian_focus_geometry():
    for w0, lam, key in [(50.0, 800.0, "rayleigh_range_focus_mm"), (80.0, 1030.0, "rayleigh_range_volume_mm")]:
        zr_mm = math.pi * w0 ** 2 / (lam * 1e-3) * 1e-3
        assert abs(zr_mm - G[key]["value"]) < G[key]["tol"]
    e0, ph, r, z = ti.gaussian_focus(32, 32, 50.0, 800.0, 2e14)
    assert e0.shape == (1024,)
    # on axis at focus: peak amplitude, zero phase; amplitude falls off radially and along z
    centre = np.argmin(r ** 2 + z ** 2)
    assert abs(z[centre]) > 0  # 32 z samples: focus lies between two planes
    assert np.max(e0) <= ti.field_amplitude(2e14) + 1e-15
    onaxis = e0[r == 0]
    assert np.argmax(onaxis) in (15, 16)


def test_pulse_shape_and_support():
    e = ti.sin2_pulse(0.05, 0.057, 10, 0.05)
    assert e.shape == (22048,)
    assert e[0] == 0.0 and abs(e[-1]) < 1e-6
    assert abs(np.max(np.abs(e)) - 0.05) < 1e-3


def test_uneven_sizes_and_seeds():
    w = ti.cfg3_uneven(256)
    n = np.array(w.n_per)
    assert n.min() >= 2048 and n.max() <= 16384 and np.all(n % 256 == 0)
    assert w.nt == ti.n_steps(0.0351, 12, 0.025)
    ww = ti.cfg3_uneven(256, wide=True)
    assert np.array(ww.n_per).max() > 8192
    assert np.array_equal(ti.cfg3_uneven(256).e0, w.e0)      # seeded


def test_adjoint_workload_amplitudes():
    w = ti.cfg4_adjoint()
    assert w.batch == 256 and np.all((w.e0 >= 0.05) & (w.e0 <= 0.075))


def test_time_windows_hold_the_full_series_samples():
    """A window i0..i0+nt of the field is bitwise the same samples as the
    full series (the benchmark chains time segments of one pulse)."""
    w = ti.cfg5_volume(2, 4)
    full = w.efield()
    for i0, nt in [(0, 100), (10653, 10653), (w.nt - 37, 37)]:
        win = w.efield(i0=i0, nt=nt)
        assert win.shape == (w.batch, nt + 1)
        assert np.array_equal(win, full[:, i0:i0 + nt + 1])
    rest = w.efield(i0=w.nt - 5)
    assert np.array_equal(rest, full[:, -6:])
    # past the end of the pulse the field is zero
    assert np.all(w.efield(i0=w.nt, nt=50)[:, 1:] == 0.0)


def test_subset_keeps_rows_and_fields():
    w = ti.cfg5_volume(4, 8)
    rows = [5, 0, 31]
    sub = w.subset(rows)
    assert sub.batch == 3 and sub.nt == w.nt and sub.dx == w.dx
    assert np.array_equal(sub.efield(nt=50), w.efield(rows=rows, nt=50))
    assert np.array_equal(sub.meta["r_um"], w.meta["r_um"][rows])
    assert sub.meta["band"] == w.meta["band"]
