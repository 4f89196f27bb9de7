"""Pins of the oracle's far-field diffraction integral (section "XUV
Propagation (Spectral Approach)", homogeneous medium) and of the band
spectrum's adjoint, against closed forms and invariants:

* a Gaussian source sheet: the radial integral with the J0 kernel and the
  paraxial phase has the closed form int_0^inf exp(-a r^2) J0(b r) r dr =
  exp(-b^2/(4a))/(2a) (Re a > 0), evaluated here with a Gauss-Legendre rule;
* longitudinal phase matching of an on-axis line of emitters: the coherent sum
  is a geometric series with a closed-form modulus;
* the adjoint identity Re<K s, e> = Re<s, K^H e>;
* the band adjoint against the exact gradient of a linear functional and
  against the yield gradient of harmonic_yield."""
import numpy as np
import pytest

import oracle


def _gauss_sheet(k, w, d, rho_obs, n=240, r_max=9.0):
    x, g = np.polynomial.legendre.leggauss(n)
    r = 0.5 * r_max * (x + 1.0)
    wr = 0.5 * r_max * g * r                         # rho' drho'
    src = np.exp(-(r / w) ** 2)[:, None] * np.ones((1, len(k)))
    E = oracle.far_field(src, r, [0.0], wr, k, rho_obs, d)
    return E


@pytest.mark.parametrize("k", [4.0, 10.0, 25.0])
def test_gaussian_sheet_matches_hankel_closed_form(k):
    w, d = 1.0, 50.0
    rho = np.array([0.0, 0.7, 3.0, 8.0])
    E = _gauss_sheet(np.array([k]), w, d, rho)[:, 0]
    a = 1.0 / w ** 2 - 1j * k / (2.0 * d)
    b = k * rho / d
    ref = -np.exp(1j * k * d) / (4 * np.pi) * np.exp(1j * k * rho ** 2 / (2 * d)) / d \
        * np.exp(-b ** 2 / (4 * a)) / (2 * a)
    assert np.max(np.abs(E - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_on_axis_line_phase_matching():
    """Emitters on the axis at z'_j = j h with S_j = exp(i kappa z'_j), seen
    from far away: |E| = |sum_j exp(i (kappa - k) z'_j)| / (4 pi d), a
    geometric series; it peaks when kappa = k (phase matching)."""
    k, h, n = 3.0, 0.05, 400
    z = h * np.arange(n)
    d0 = 1e9
    for kappa in (3.0, 2.9, 3.2):
        src = np.exp(1j * kappa * z)[None, :, None]           # one radial node
        E = oracle.far_field(src.reshape(n, 1), [0.0], z, np.ones(n), [k], [0.0], d0)[0, 0]
        delta = kappa - k
        s = n if delta == 0.0 else abs(np.sin(n * delta * h / 2) / np.sin(delta * h / 2))
        # 1/d_j varies by at most n h / d0 across the line
        assert abs(abs(E) * 4 * np.pi * d0 - s) <= 1e-6 * n
    E_pm = oracle.far_field(np.exp(1j * k * z).reshape(n, 1), [0.0], z, np.ones(n), [k], [0.0], d0)
    E_mm = oracle.far_field(np.exp(1j * 0.9 * k * z).reshape(n, 1), [0.0], z, np.ones(n), [k], [0.0], d0)
    assert abs(E_pm[0, 0]) > 10 * abs(E_mm[0, 0])


def test_far_field_adjoint_identity():
    rng = np.random.default_rng(4)
    r = np.linspace(0.0, 2.0, 5)
    z = np.linspace(-1.0, 1.0, 7)
    wts = rng.uniform(0.5, 1.5, 35)
    kw = np.array([5.0, 7.5, 11.0])
    ro = np.array([0.0, 0.3, 1.1])
    s = rng.standard_normal((35, 3)) + 1j * rng.standard_normal((35, 3))
    e = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    lhs = np.real(np.vdot(e, oracle.far_field(s, r, z, wts, kw, ro, 40.0)))
    rhs = np.real(np.vdot(oracle.far_field_adjoint(e, r, z, wts, kw, ro, 40.0), s))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_band_adjoint_is_the_gradient_of_a_linear_functional():
    rng = np.random.default_rng(5)
    nt, dt, om = 300, 0.05, 0.25
    a = rng.standard_normal(nt + 1)
    kb, A = oracle.band_amplitudes(a, dt, om, 3, 9)
    c = rng.standard_normal(len(kb)) + 1j * rng.standard_normal(len(kb))
    g = oracle.band_adjoint(c, nt + 1, dt, kb)[0]
    # l(a) = Re sum_k conj(c_k) A_k(a) is linear in a: l(a) = g . a exactly
    assert abs(np.real(np.vdot(c, A[0])) - g @ a) <= 1e-12 * np.abs(g).sum() * np.abs(a).max()
    # yield: dl/dA = 2 domega A, which must reproduce harmonic_yield's gradient
    _, abar = oracle.harmonic_yield(a, dt, om, 3, 9)
    dw = 2 * np.pi / ((nt + 1) * dt)
    g2 = oracle.band_adjoint(2 * dw * A, nt + 1, dt, kb)
    assert np.allclose(g2, abar, rtol=0, atol=1e-13 * np.abs(abar).max())
