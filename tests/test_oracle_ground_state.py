"""Pins of the oracle's imaginary-time ground state and soft-core fit against a
dense symmetric eigensolver, the Hellmann-Feynman theorem and monotonicity."""
import numpy as np
import pytest

import oracle
import tdse_inputs as ti
from dense_reference import dense_h, grid_x


@pytest.mark.parametrize("n,dx,a", [(512, 0.2, 1.18917), (1024, 0.15, 0.9), (301, 0.3, 2.0)])
def test_ground_state_is_lowest_dense_eigenpair(n, dx, a):
    h, _ = dense_h(n, dx, a)
    w, v = np.linalg.eigh(h)
    psi, e, _ = oracle.ground_state(n, dx, a, dtau=1.0, tol=1e-13)
    assert abs(e - w[0]) < 1e-12
    ref = v[:, 0] / np.sqrt(dx)
    ref *= np.sign(ref[n // 2])
    assert np.max(np.abs(psi.imag)) == 0.0
    assert psi.real[n // 2] > 0
    assert np.max(np.abs(psi.real - ref)) < 1e-9 * np.max(np.abs(ref))
    assert abs(dx * np.sum(np.abs(psi) ** 2) - 1.0) < 1e-13


def test_fixed_point_does_not_depend_on_dtau():
    p1, e1, _ = oracle.ground_state(400, 0.2, 1.3, dtau=0.3, tol=1e-13)
    p2, e2, _ = oracle.ground_state(400, 0.2, 1.3, dtau=2.0, tol=1e-13)
    assert abs(e1 - e2) < 1e-13
    assert np.max(np.abs(p1 - p2)) < 1e-10


def test_ground_state_energy_increases_with_a_hellmann_feynman():
    """dE_g/da = <psi| dV/da |psi> = <a (x^2+a^2)^-3/2> > 0."""
    n, dx, a, h = 800, 0.2, 1.2, 1e-4
    _, ep, _ = oracle.ground_state(n, dx, a + h)
    _, em, _ = oracle.ground_state(n, dx, a - h)
    psi, _, _ = oracle.ground_state(n, dx, a)
    x = grid_x(n, dx)
    hf = dx * np.sum(np.abs(psi) ** 2 * a * (x ** 2 + a ** 2) ** -1.5)
    fd = (ep - em) / (2 * h)
    assert fd > 0
    assert abs(fd - hf) / hf < 1e-4   # the Numerov kinetic term makes HF approximate


def test_soft_core_fit_reaches_argon_ip():
    """a with E_g(a) = -Ip (Ip = 0.5792, argon) on the single-system grid."""
    a, e = oracle.soft_core_for_ip(ti.IP_ARGON, 2048, 0.2, tol=1e-13)
    assert abs(e + ti.IP_ARGON) < 1e-13
    h, _ = dense_h(2048, 0.2, a)
    w = np.linalg.eigvalsh(h)
    assert abs(w[0] + ti.IP_ARGON) < 1e-12
