"""Pins of the oracle's electron energy distribution P(E) =
(eps/pi) ||(E - i eps - H0)^{-1} psi||^2 (dx-weighted norm), against the
spectral theorem with the dense symmetric Numerov Hamiltonian, the exact
Lorentzian peak of an eigenstate, and the sum rule int P dE = ||psi||^2."""
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
