"""Pins of the oracle's electron energy distribution P(E) =
(eps/pi) ||(E - i eps - H0)^{-1} psi||^2 (dx-weighted norm), against the
spectral theorem with the dense symmetric Numerov Hamiltonian, the exact
Lorentzian peak of an eigenstate, and the sum rule int P dE = ||psi||^2; and
of the energy integral (the ionisation probability) against the closed-form
integral of that Lorentzian and the exactness of the trapezoid rule on
piecewise-linear data."""
import numpy as np

import oracle
from dense_reference import dense_h


def test_matches_the_spectral_sum_of_the_dense_hamiltonian():
    n, dx, a, eps = 160, 0.3, 1.1, 0.05
    h, x = dense_h(n, dx, a)
    lam, vec = np.linalg.eigh(h)
    rng = np.random.default_rng(2)
    psi = np.exp(-(x - 1.0) ** 2 / 4.0) * np.exp(0.8j * x) + 0.2 * rng.standard_normal(n)
    psi /= np.sqrt(dx * np.sum(np.abs(psi) ** 2))
    c = vec.T @ psi
    energies = np.linspace(-0.8, 3.0, 37)
    ref = np.array([eps / np.pi * dx * np.sum(np.abs(c) ** 2 / ((e - lam) ** 2 + eps ** 2))
                    for e in energies])
    got = oracle.energy_spectrum(psi, energies, eps, dx, a)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(ref)


def test_eigenstate_gives_a_lorentzian_of_height_one_over_pi_eps():
    n, dx, a, eps = 256, 0.2, 1.2, 1e-3
    psi, e_g, _ = oracle.ground_state(n, dx, a, dtau=0.5)
    p = oracle.energy_spectrum(psi, [e_g, e_g + eps, e_g + 3 * eps], eps, dx, a)
    lor = 1.0 / (np.pi * eps) / (1.0 + np.array([0.0, 1.0, 9.0]))
    assert np.max(np.abs(p - lor) / lor) < 1e-7


def test_sum_rule():
    n, dx, a, eps = 200, 0.25, 1.1, 0.02
    h, x = dense_h(n, dx, a)
    lam = np.linalg.eigvalsh(h)
    psi = np.exp(-x ** 2) * (1 + 0.5 * x)
    psi = psi / np.sqrt(dx * np.sum(np.abs(psi) ** 2))
    e = np.linspace(lam[0] - 40 * eps, lam[-1] + 40 * eps, 60001)
    p = oracle.energy_spectrum(psi, e, eps, dx, a)
    total = np.trapezoid(p, e)
    # the Lorentzian tails beyond the range hold at most 2 eps / (pi 40 eps)
    assert abs(total - 1.0) < 2.0 / (np.pi * 40) + 1e-6


def test_energy_integral_is_exact_on_linear_pieces_and_respects_the_threshold():
    # the trapezoid rule integrates a piecewise-linear function exactly; only
    # the intervals whose two ends lie at or above e_lo count
    e = np.array([-1.0, -0.25, 0.0, 0.5, 2.0, 3.5])
    p = np.array([[7.0, 1.0, 2.0, 3.0, 0.0, 6.0],
                  [1.0, 1.0, 1.0, 1.0, 1.0, 1.0]])
    got = oracle.energy_integral(e, p, 0.0)
    # row 0 above 0: 0.5*(2+3)*0.5 + 1.5*(3+0)/2 + 1.5*(0+6)/2
    assert np.allclose(got, [1.25 + 2.25 + 4.5, 3.5], rtol=0, atol=1e-15)
    assert np.allclose(oracle.energy_integral(e, p, -np.inf), [0.75 * 4.0 + 0.25 * 1.5 + 8.0, 4.5],
                       rtol=0, atol=1e-15)
    assert np.allclose(oracle.energy_integral(e, p, 10.0), [0.0, 0.0])


def test_ionisation_of_an_eigenstate_is_the_lorentzian_tail():
    # P(E) of an eigenstate with norm 1 is (eps/pi) / ((E - E_g)^2 + eps^2), so
    # its integral over [0, E_max] is (arctan((E_max - E_g)/eps) - arctan(-E_g/eps))/pi;
    # the trapezoid error is at most h^2 (E_max) max|P''| / 12
    n, dx, a, eps = 256, 0.2, 1.2, 0.05
    psi, e_g, _ = oracle.ground_state(n, dx, a, dtau=0.5)
    e = np.linspace(0.0, 2.0, 2001)
    got = oracle.ionisation_probability(psi, e, eps, dx, a)
    ref = (np.arctan((2.0 - e_g) / eps) - np.arctan(-e_g / eps)) / np.pi
    h = e[1] - e[0]
    d2max = 2.0 * eps / np.pi / e_g ** 4 * 3.0  # bound on |P''| for E >= 0 > E_g + eps
    assert abs(got - ref) <= h * h * 2.0 * d2max / 12.0 + 1e-9 * ref
    assert 0.0 < got < 0.1
