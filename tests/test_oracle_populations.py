"""Pins of oracle.populations (ground-state and volumetric populations of a
wavefunction, section "Microscopic Response in XUV regime (TDSE)"): the
normalised ground state has population 1, a state of the other parity 0, a
superposition |c0|^2; the volumetric population of a Gaussian is the normal
distribution's mass over the covered cells, and covers the norm for a radius
past the box."""
import math

import numpy as np

import oracle


def _ground(n=512, dx=0.2, a=1.1):
    psi0, _, _ = oracle.ground_state(n, dx, a, dtau=1.0, tol=1e-12)
    return psi0, dx


def test_ground_state_population_is_one_and_volume_is_the_norm():
    psi0, dx = _ground()
    gs, vol = oracle.populations(psi0, psi0, dx, radius=1e9)
    assert abs(gs - 1.0) < 1e-12
    assert abs(vol - 1.0) < 1e-12
    # a phase on either state leaves the population unchanged
    gs2, _ = oracle.populations(np.exp(0.7j) * psi0, np.exp(-1.9j) * psi0, dx, radius=0.0)
    assert abs(gs2 - gs) < 1e-13


def test_odd_state_and_superposition():
    psi0, dx = _ground()
    n = psi0.shape[0]
    x = (np.arange(n) - 0.5 * (n - 1)) * dx
    psi1 = x * psi0
    psi1 /= math.sqrt(dx * np.sum(np.abs(psi1) ** 2))
    gs_odd, _ = oracle.populations(psi1, psi0, dx, radius=1.0)
    assert gs_odd < 1e-24
    c0, c1 = 0.6 * np.exp(0.3j), 0.8 * np.exp(-1.1j)
    gs, vol = oracle.populations(c0 * psi0 + c1 * psi1, psi0, dx, radius=1e9)
    assert abs(gs - 0.36) < 1e-12
    assert abs(vol - 1.0) < 1e-12
    # swapping the roles of psi and phi gives the same population
    gs_sw, _ = oracle.populations(psi0, c0 * psi0 + c1 * psi1, dx, radius=0.0)
    assert abs(gs_sw - gs) < 1e-12


def test_volumetric_population_of_a_gaussian():
    n, dx, sigma = 2001, 0.05, 3.0
    x = (np.arange(n) - 0.5 * (n - 1)) * dx
    psi = (2 * math.pi * sigma ** 2) ** -0.25 * np.exp(-x ** 2 / (4 * sigma ** 2)) * np.exp(0.4j * x)
    prev = 0.0
    for radius in (0.01, 1.013, 2.537, 6.02):
        _, vol = oracle.populations(psi, psi, dx, radius)
        inside = np.abs(x) <= radius
        # the included cells span [-R, R], R = last included point + dx / 2
        R = x[inside].max() + 0.5 * dx
        assert abs(vol - math.erf(R / (sigma * math.sqrt(2.0)))) < 2e-5
        assert vol >= prev
        prev = vol
