"""CPU oracle for the 1D-TDSE microscopic step (arXiv 2507.04115).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, loads or calls it, and the
two share no code: the numerical core is the plain C file ``tdse_ref.c``
(serial, fp64, Thomas algorithm, matrices rebuilt from their definitions),
the harmonic-yield loss below is a direct discrete Fourier sum in numpy, and
the far-field diffraction integral is a direct sum over the medium in numpy
(scipy's J0).

Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` against closed forms, dense textbook linear algebra
(numpy/scipy), physical invariants or finite differences; none is "parity
unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtdse_ref.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433 (local build of the C oracle)

        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    d, i = ctypes.c_double, ctypes.c_int
    lib.tdse_ref_grid.argtypes = [i, d, d, d, _dp, _dp, _dp]
    lib.tdse_ref_mask.argtypes = [i, d, d, d, _dp]
    lib.tdse_ref_propagate.argtypes = [i, d, d, d, d, d, d, i, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.tdse_ref_propagate_batch.argtypes = [i, _ip, _i64p, d, d, d, d, d, d, i, _dp, _dp, _dp,
                                        _dp, _dp, i]
    lib.tdse_ref_ground_state.argtypes = [i, d, d, d, d, i, d, _dp, _dp, _ip]
    lib.tdse_ref_soft_core_for_ip.argtypes = [d, i, d, d, d, i, d, d, d, _dp, _dp]
    lib.tdse_ref_adjoint.argtypes = [i, d, d, d, d, d, d, i, _dp, _dp, _dp, i, _dp, _dp]
    lib.tdse_ref_step.argtypes = [i, d, d, d, d, d, d, d, _dp]
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _check(st, what):
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def _c128(psi, n):
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    if psi.shape != (n,):
        raise ValueError(f"psi must have shape ({n},), got {psi.shape}")
    return psi


# --------------------------------------------------------------------------
# grid, potential, mask
# --------------------------------------------------------------------------

def grid(n, dx, a=1.0, z=1.0):
    """x_j, V_j = -z/sqrt(x^2+a^2) and dV/dx on the N-point centred grid."""
    x = np.empty(n)
    v = np.empty(n)
    dv = np.empty(n)
    _check(_load().tdse_ref_grid(n, dx, a, z, _ptr(x), _ptr(v), _ptr(dv)), "tdse_ref_grid")
    return x, v, dv


def mask(n, dx, frac=0.1, power=0.125):
    m = np.empty(n)
    _check(_load().tdse_ref_mask(n, dx, frac, power, _ptr(m)), "tdse_ref_mask")
    return m


# --------------------------------------------------------------------------
# propagation
# --------------------------------------------------------------------------

def step(psi, dx, dt, a, z, e, mask_frac=0.0, mask_pow=0.125):
    """One Crank-Nicolson + field step psi^(i) -> psi^(i+1) with E(t_i) = e."""
    n = len(psi)
    out = _c128(psi, n).copy()
    _check(_load().tdse_ref_step(n, dx, dt, a, z, mask_frac, mask_pow, e,
                            out.ctypes.data_as(_dp)), "tdse_ref_step")
    return out


def propagate(efield, psi0, dx, dt, a, z=1.0, mask_frac=0.1, mask_pow=0.125,
              want_psi=False):
    """Forward solve. Returns dict with accel, xexp, norm (nt+1 samples each)
    and optionally psi_final."""
    efield = np.ascontiguousarray(efield, dtype=np.float64)
    nt = efield.shape[0] - 1
    n = len(psi0)
    psi0 = _c128(psi0, n)
    acc = np.empty(nt + 1)
    xe = np.empty(nt + 1)
    nr = np.empty(nt + 1)
    pf = np.empty(n, dtype=np.complex128) if want_psi else None
    st = _load().tdse_ref_propagate(n, dx, dt, a, z, mask_frac, mask_pow, nt, _ptr(efield),
                               psi0.ctypes.data_as(_dp), _ptr(acc), _ptr(xe), _ptr(nr),
                               pf.ctypes.data_as(_dp) if pf is not None else None)
    _check(st, "tdse_ref_propagate")
    out = {"accel": acc, "xexp": xe, "norm": nr}
    if want_psi:
        out["psi_final"] = pf
    return out


def propagate_batch(efield, psi0_list, dx, dt, a, z=1.0, mask_frac=0.1, mask_pow=0.125,
                    nthreads=1):
    """Forward solve of a batch on host threads. efield: [P, nt+1]."""
    efield = np.ascontiguousarray(efield, dtype=np.float64)
    batch, ntp1 = efield.shape
    n_per = np.array([len(p) for p in psi0_list], dtype=np.int32)
    off = np.zeros(batch + 1, dtype=np.int64)
    off[1:] = np.cumsum(n_per)
    psi0 = np.ascontiguousarray(np.concatenate([np.asarray(p, np.complex128)
                                                for p in psi0_list]))
    acc = np.empty((batch, ntp1))
    xe = np.empty((batch, ntp1))
    nr = np.empty((batch, ntp1))
    st = _load().tdse_ref_propagate_batch(batch, n_per.ctypes.data_as(_ip), off.ctypes.data_as(_i64p),
                                     dx, dt, a, z, mask_frac, mask_pow, ntp1 - 1, _ptr(efield),
                                     psi0.ctypes.data_as(_dp), _ptr(acc), _ptr(xe), _ptr(nr),
                                     nthreads)
    _check(st, "tdse_ref_propagate_batch")
    return {"accel": acc, "xexp": xe, "norm": nr}


# --------------------------------------------------------------------------
# ground state and soft-core fit
# --------------------------------------------------------------------------

def ground_state(n, dx, a, z=1.0, dtau=1.0, max_iter=20000, tol=1e-13):
    """Imaginary-time relaxation. Returns (psi0 complex128, energy, iterations)."""
    psi = np.empty(n, dtype=np.complex128)
    e = ctypes.c_double()
    it = ctypes.c_int()
    st = _load().tdse_ref_ground_state(n, dx, a, z, dtau, max_iter, tol, psi.ctypes.data_as(_dp),
                                  ctypes.byref(e), ctypes.byref(it))
    _check(st, "tdse_ref_ground_state")
    return psi, e.value, it.value


def soft_core_for_ip(ip, n, dx, dtau=1.0, gs_tol=1e-13, gs_max_iter=20000, tol=1e-13,
                     a_lo=0.5, a_hi=3.0):
    """Bisection on a so that the ground-state energy equals -ip.
    Returns (a, E_g(a))."""
    a = ctypes.c_double()
    e = ctypes.c_double()
    st = _load().tdse_ref_soft_core_for_ip(ip, n, dx, dtau, gs_tol, gs_max_iter, tol, a_lo, a_hi,
                                      ctypes.byref(a), ctypes.byref(e))
    _check(st, "tdse_ref_soft_core_for_ip")
    return a.value, e.value


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

def adjoint(efield, psi0, abar, dx, dt, a, z=1.0, mask_frac=0.1, mask_pow=0.125, k=256):
    """Gradient dl/dE_i of a loss l(a_0..a_nt) given abar_i = dl/da_i.
    Returns (grad, accel)."""
    efield = np.ascontiguousarray(efield, dtype=np.float64)
    abar = np.ascontiguousarray(abar, dtype=np.float64)
    nt = efield.shape[0] - 1
    if abar.shape != efield.shape:
        raise ValueError("abar must match efield")
    n = len(psi0)
    psi0 = _c128(psi0, n)
    grad = np.empty(nt + 1)
    acc = np.empty(nt + 1)
    st = _load().tdse_ref_adjoint(n, dx, dt, a, z, mask_frac, mask_pow, nt, _ptr(efield),
                             psi0.ctypes.data_as(_dp), _ptr(abar), k, _ptr(grad), _ptr(acc))
    _check(st, "tdse_ref_adjoint")
    return grad, acc


# --------------------------------------------------------------------------
# harmonic-yield loss (direct band DFT)
# --------------------------------------------------------------------------

def band_bins(ntp1, dt, omega0, h_lo, h_hi):
    """Indices k with h_lo*omega0 <= omega_k <= h_hi*omega0, where
    omega_k = 2 pi k / (ntp1 dt) are the DFT frequencies of ntp1 samples."""
    dw = 2.0 * np.pi / (ntp1 * dt)
    k = np.arange(ntp1 // 2 + 1)
    w = k * dw
    return k[(w >= h_lo * omega0) & (w <= h_hi * omega0)]


def harmonic_yield(accel, dt, omega0, h_lo, h_hi):
    """Windowed harmonic yield of each row of ``accel`` ([P, nt+1]) and its
    gradient with respect to the samples.

      w_i   = sin^2(pi i / nt)                       (symmetric Hann window)
      A_k   = dt sum_i w_i a_i exp(-i omega_k t_i),  t_i = i dt
      l     = sum_{k in band} domega |A_k|^2,        domega = 2 pi / ((nt+1) dt)
      dl/da_i = 2 domega dt w_i sum_{k in band} Re(conj(A_k) exp(-i omega_k t_i))

    Returns (l per row, dl/da [P, nt+1])."""
    accel = np.atleast_2d(np.asarray(accel, dtype=np.float64))
    ntp1 = accel.shape[1]
    nt = ntp1 - 1
    i = np.arange(ntp1)
    w = np.sin(np.pi * i / nt) ** 2
    kb = band_bins(ntp1, dt, omega0, h_lo, h_hi)
    dw = 2.0 * np.pi / (ntp1 * dt)
    # exp(-i omega_k t_i) with omega_k t_i = 2 pi (k i mod ntp1) / ntp1
    ph = np.exp(-2j * np.pi * (np.outer(kb, i) % ntp1) / ntp1)  # [K, ntp1]
    amp = dt * (accel * w) @ ph.T                                # [P, K]
    loss = dw * np.sum(np.abs(amp) ** 2, axis=1)
    abar = 2.0 * dw * dt * w * np.real(np.conj(amp) @ ph)        # [P, ntp1]
    return loss, abar


def band_amplitudes(accel, dt, omega0, h_lo, h_hi):
    """(band bins k, A [P, K]) with A_k = dt sum_i w_i a_i exp(-i omega_k t_i),
    the windowed spectrum of ``harmonic_yield`` on its band."""
    accel = np.atleast_2d(np.asarray(accel, dtype=np.float64))
    ntp1 = accel.shape[1]
    i = np.arange(ntp1)
    w = np.sin(np.pi * i / (ntp1 - 1)) ** 2
    kb = band_bins(ntp1, dt, omega0, h_lo, h_hi)
    ph = np.exp(-2j * np.pi * (np.outer(kb, i) % ntp1) / ntp1)
    return kb, dt * (accel * w) @ ph.T


def band_adjoint(amp_bar, ntp1, dt, kb):
    """Gradient of a real loss with respect to the samples a_i, given
    amp_bar_k = dl/dRe A_k + i dl/dIm A_k for the band amplitudes above:
    dl/da_i = dt w_i sum_k Re(conj(amp_bar_k) exp(-i omega_k t_i))."""
    amp_bar = np.atleast_2d(np.asarray(amp_bar, dtype=np.complex128))
    i = np.arange(ntp1)
    w = np.sin(np.pi * i / (ntp1 - 1)) ** 2
    ph = np.exp(-2j * np.pi * (np.outer(kb, i) % ntp1) / ntp1)
    return dt * w * np.real(np.conj(amp_bar) @ ph)


# --------------------------------------------------------------------------
# far field of the XUV emission (diffraction integral over the medium)
# --------------------------------------------------------------------------

def far_field_kernel(rho_src, z_src, weights, kw, rho_obs, z_obs):
    """K[q, m, p]: the propagator of the homogeneous-medium diffraction
    integral (section "XUV Propagation (Spectral Approach)", Eq. of the
    far field in a homogeneous generating medium), with mu0 left to the
    caller:

      E(rho_m, z, omega_q) = -(exp(i k z) / (4 pi)) sum_{p=(i,j)} w_p
            exp(-i k z'_j) exp(i k rho_m^2 / (2 d_j)) / d_j
            exp(i k rho'_i^2 / (2 d_j)) J0(k rho_m rho'_i / d_j) S_p(omega_q),

    k = kw[q], d_j = z - z'_j, p = i * n_z + j; w_p are the quadrature
    weights of the rho' drho' dz' integral times the gas density."""
    from scipy.special import j0

    rho_src = np.asarray(rho_src, np.float64)
    z_src = np.asarray(z_src, np.float64)
    R = np.repeat(rho_src, len(z_src))            # rho'_i of p
    Z = np.tile(z_src, len(rho_src))              # z'_j of p
    W = np.asarray(weights, np.float64).ravel()
    d = z_obs - Z
    K = np.empty((len(kw), len(rho_obs), len(R)), np.complex128)
    for q, k in enumerate(kw):
        for m, r in enumerate(rho_obs):
            phase = k * (R ** 2 + r ** 2) / (2.0 * d) - k * Z
            K[q, m] = -np.exp(1j * k * z_obs) / (4.0 * np.pi) * W / d * np.exp(1j * phase) \
                * j0(k * r * R / d)
    return K


def far_field(amp, rho_src, z_src, weights, kw, rho_obs, z_obs):
    """Far field E [M, Q] of the source spectra amp [P, Q] (see
    far_field_kernel)."""
    K = far_field_kernel(rho_src, z_src, weights, kw, rho_obs, z_obs)
    amp = np.asarray(amp, np.complex128)
    return np.stack([K[q] @ amp[:, q] for q in range(len(kw))], axis=1)


def far_field_adjoint(field_bar, rho_src, z_src, weights, kw, rho_obs, z_obs):
    """amp_bar [P, Q] = sum_m conj(K[q, m, p]) field_bar[m, q]: the gradient
    of a real loss with respect to the source spectra, given its gradient
    with respect to the far field (same complex convention as band_adjoint)."""
    K = far_field_kernel(rho_src, z_src, weights, kw, rho_obs, z_obs)
    fb = np.asarray(field_bar, np.complex128)
    return np.stack([np.conj(K[q]).T @ fb[:, q] for q in range(len(kw))], axis=1)


# --------------------------------------------------------------------------
# electron energy distribution (resolvent of the field-free Hamiltonian)
# --------------------------------------------------------------------------

def energy_spectrum(psi, energies, eps, dx, a, z=1.0):
    """P(E) = (eps / pi) dx sum_j |phi_j|^2 with (E - i eps - H0) phi = psi
    (section "Analysing the Time-Dependent Electron Energy Density": the
    resolvent norm, the inverse taken in the solver's Numerov form).  With
    H0 = M2^{-1}(-D2/2) + V the system is multiplied by M2:
      ((E - i eps) M2 - A) phi = M2 psi,   A = -D2/2 + M2 diag(V),
    a tridiagonal system solved here with scipy's banded solver.  The factor
    1/(pi eps) makes int P dE equal dx sum |psi|^2."""
    from scipy.linalg import solve_banded

    psi = np.asarray(psi, np.complex128)
    n = len(psi)
    _, v, _ = grid(n, dx, a, z)
    mpsi = 10.0 * psi
    mpsi[1:] += psi[:-1]
    mpsi[:-1] += psi[1:]
    mpsi /= 12.0
    out = np.empty(len(energies))
    for q, e in enumerate(energies):
        ec = e - 1j * eps
        ab = np.zeros((3, n), np.complex128)
        ab[1] = ec * 10.0 / 12.0 - (1.0 / dx ** 2 + 10.0 / 12.0 * v)     # T[j, j]
        ab[0, 1:] = ec / 12.0 + 0.5 / dx ** 2 - v[1:] / 12.0           # T[j, j+1]
        ab[2, :-1] = ec / 12.0 + 0.5 / dx ** 2 - v[:-1] / 12.0         # T[j+1, j]
        phi = solve_banded((1, 1), ab, mpsi)
        out[q] = eps / np.pi * dx * np.sum(np.abs(phi) ** 2)
    return out


def energy_integral(energies, spectrum, e_lo):
    """int_{E >= e_lo} P(E) dE by the trapezoid rule over the grid points
    E_e >= e_lo (section "Analysing the Time-Dependent Electron Energy
    Density": integrated over the energies above the ionisation threshold,
    e_lo = 0, the distribution of psi(t) gives the time-dependent ionisation
    probability).  energies increasing; spectrum [..., n_energy]."""
    e = np.asarray(energies, np.float64)
    p = np.asarray(spectrum, np.float64)
    total = np.zeros(p.shape[:-1])
    for q in range(len(e) - 1):
        if e[q] >= e_lo and e[q + 1] >= e_lo:
            total = total + 0.5 * (e[q + 1] - e[q]) * (p[..., q] + p[..., q + 1])
    return total


def ionisation_probability(psi, energies, eps, dx, a, z=1.0):
    """The time-dependent ionisation probability of a state: its energy
    distribution integrated over E >= 0 on the given grid."""
    return energy_integral(energies, energy_spectrum(psi, energies, eps, dx, a, z), 0.0)


# --------------------------------------------------------------------------
# driver-field resampling (Fourier zero-padding)
# --------------------------------------------------------------------------

def resample_field(e_coarse, dt_coarse, dt, nt):
    """Fine samples E(i dt), i = 0..nt, of fields given at M coarse samples
    (spacing dt_coarse, the first one taken as t = 0: the time-axis shift of
    section "1D-TSDE Implementation (CTDSE)"), by Fourier zero-padding: the
    trigonometric interpolant of period T = M dt_coarse,
      E(t) = (1/M) [X_0 + sum_{0<k<M/2} 2 Re(X_k exp(2 pi i k t / T))
                    + (M even) Re(X_{M/2}) cos(pi M t / T)],
    with X the DFT of the coarse samples, evaluated directly.  T/dt must be
    an integer (the padded length) no smaller than nt + 1."""
    e = np.atleast_2d(np.asarray(e_coarse, np.float64))
    M = e.shape[1]
    T = M * dt_coarse
    X = np.fft.rfft(e, axis=1)
    t = dt * np.arange(nt + 1)
    out = np.repeat(X[:, :1].real, nt + 1, axis=1)
    for k in range(1, (M + 1) // 2):
        out = out + 2.0 * np.real(X[:, k:k + 1] * np.exp(2j * np.pi * k * t / T)[None, :])
    if M % 2 == 0:
        out = out + X[:, M // 2:M // 2 + 1].real * np.cos(np.pi * M * t / T)[None, :]
    return out / M


def gabor(accel, dt, t_centres, omegas, sigma):
    """Gabor transform of the source term: G[b, c, w] =
    |dt sum_i a_b,i exp(-(t_i - t_c)^2 / (2 sigma^2)) exp(-i omega_w t_i)|^2,
    t_i = i dt, summed over every sample."""
    accel = np.atleast_2d(np.asarray(accel, np.float64))
    t = dt * np.arange(accel.shape[1])
    ph = np.exp(-1j * np.outer(omegas, t))                           # [W, nt+1]
    out = np.empty((accel.shape[0], len(t_centres), len(omegas)))
    for c, tc in enumerate(t_centres):
        win = np.exp(-(t - tc) ** 2 / (2.0 * sigma ** 2))
        out[:, c, :] = np.abs(dt * (accel * win) @ ph.T) ** 2
    return out


def populations(psi, phi, dx, radius):
    """Ground-state and volumetric populations of a wavefunction (section
    "Microscopic Response in XUV regime (TDSE)", the analyses of psi listed
    after the dipole acceleration): (|dx <phi, psi>|^2,
    dx sum_{|x_j| <= radius} |psi_j|^2) on the centred grid
    x_j = (j - (n-1)/2) dx."""
    psi = np.asarray(psi, np.complex128)
    phi = np.asarray(phi, np.complex128)
    n = psi.shape[0]
    x = (np.arange(n) - 0.5 * (n - 1)) * dx
    gs = abs(dx * np.vdot(phi, psi)) ** 2
    inside = np.abs(x) <= radius
    vol = dx * float(np.sum(np.abs(psi[inside]) ** 2))
    return gs, vol
