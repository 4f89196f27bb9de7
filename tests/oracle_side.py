"""The oracle's side of a parity test, computed from the seeded inputs
alone: its own ground states, soft-core fits, accelerations and loss
gradients.  Nothing here takes a value from the HIP path, so a parity test
compares two computations that share only their inputs."""
import functools

import oracle


@functools.lru_cache(maxsize=None)
def ground_state(n, dx, a):
    """The oracle's ground state (imaginary-time relaxation to 1e-14)."""
    return oracle.ground_state(n, dx, a, dtau=1.0, tol=1e-14)[0]


@functools.lru_cache(maxsize=None)
def soft_core(ip, dx, n=2048):
    """The oracle's soft-core parameter for the ionisation potential ip."""
    return oracle.soft_core_for_ip(ip, n, dx, dtau=1.0)[0]


def propagate(efield_row, n, dx, dt, a, **kw):
    """Forward solve from the oracle's ground state."""
    return oracle.propagate(efield_row, ground_state(n, dx, a), dx, dt, a, **kw)


def yield_gradient(efield_row, n, dx, dt, a, om, h_lo, h_hi, weight=1.0, mask_frac=0.1,
                   mask_pow=0.125, k=256):
    """(yield, dl/dE) of l = weight * harmonic yield of the row, every step on
    the oracle: forward from its ground state, loss gradient, adjoint."""
    psi0 = ground_state(n, dx, a)
    acc = oracle.propagate(efield_row, psi0, dx, dt, a, mask_frac=mask_frac,
                           mask_pow=mask_pow)["accel"]
    y, abar = oracle.harmonic_yield(acc[None, :], dt, om, h_lo, h_hi)
    g, _ = oracle.adjoint(efield_row, psi0, weight * abar[0], dx, dt, a, mask_frac=mask_frac,
                          mask_pow=mask_pow, k=k)
    return float(y[0]), g


def adjoint(efield_row, abar_row, n, dx, dt, a, mask_frac=0.1, mask_pow=0.125, k=256):
    """(grad, accel) of the oracle's adjoint for a given accel_bar row."""
    return oracle.adjoint(efield_row, ground_state(n, dx, a), abar_row, dx, dt, a,
                          mask_frac=mask_frac, mask_pow=mask_pow, k=k)
