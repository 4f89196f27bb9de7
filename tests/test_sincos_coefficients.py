"""The polynomial coefficients of the device's reduced-range sincos
(`sincos_rr` in csrc/tdse_device.hpp), read from the header and evaluated in
double precision the way the kernel evaluates them, against mpmath on
|r| <= pi/4: a mistyped or dropped coefficient fails here."""
import os
import re

import pytest

mp = pytest.importorskip("mpmath")

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2507_04115_amd", "csrc",
                   "tdse_device.hpp")


def _coefficients():
    text = open(HDR).read()
    body = text[text.index("void sincos_rr(double x"):]
    body = body[:body.index("\n}\n")]
    ks = [float(v) for v in re.findall(r"TDSE_K\(([-+0-9.eE]+)\)", body)]
    # two_over_pi, p1, p2, p3, then six for S and six for C
    assert len(ks) == 16, ks
    return ks[4:10], ks[10:16]


def _horner(coefs, t):
    p = coefs[0]
    for c in coefs[1:]:
        p = p * t + c
    return p


def test_reduced_range_sincos_polynomials():
    cs, cc = _coefficients()
    assert cs[-1] == pytest.approx(-1.0 / 6.0, rel=1e-15)
    assert cc[-1] == pytest.approx(1.0 / 24.0, rel=1e-15)
    worst_s = worst_c = 0.0
    n = 2001
    for i in range(n):
        r = -0.7853981633974483 + 1.5707963267948966 * i / (n - 1)
        t = r * r
        # the kernel's steps: sr = (ps t) r + r, cr = ((pc t) - 1/2) t + 1
        s = (_horner(cs, t) * t) * r + r
        c = (_horner(cc, t) * t - 0.5) * t + 1.0
        ref_s, ref_c = mp.sin(mp.mpf(r)), mp.cos(mp.mpf(r))
        worst_s = max(worst_s, float(abs(mp.mpf(s) - ref_s)))
        worst_c = max(worst_c, float(abs(mp.mpf(c) - ref_c)))
    assert worst_s < 2.5e-16
    assert worst_c < 2.5e-16
