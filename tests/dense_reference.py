"""Dense textbook linear algebra used only to pin the oracle.

Independent of the oracle's tridiagonal/Thomas formulation: here the
Hamiltonian is assembled as the dense symmetric matrix
H = M2^{-1}(-D2/2) + V (the operator whose Cayley transform the paper's
Crank-Nicolson step is: L^{-1} R = (I + i dt H / 2)^{-1} (I - i dt H / 2)
after multiplying both matrices by M2^{-1}) and the propagators are built
with numpy/scipy (solve, eigh, expm).
"""
import numpy as np
import scipy.linalg as sla


def grid_x(n, dx):
    return (np.arange(n) - 0.5 * (n - 1)) * dx


def dense_h(n, dx, a, z=1.0):
    x = grid_x(n, dx)
    s = np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    lap = (s - 2.0 * np.eye(n)) / dx ** 2
    m2 = np.eye(n) + dx ** 2 * lap / 12.0
    h = np.linalg.solve(m2, -0.5 * lap)
    if z != 0.0:
        h = h + np.diag(-z / np.sqrt(x ** 2 + a ** 2))
    return 0.5 * (h + h.T), x


def cayley(h, dt):
    n = h.shape[0]
    return np.linalg.solve(np.eye(n) + 0.5j * dt * h, np.eye(n) - 0.5j * dt * h)


def exact_step(h, x, dt, e):
    """exp(-i dt (H + x e)) for a constant field e."""
    return sla.expm(-1j * dt * (h + np.diag(x * e)))
