"""Seeded synthetic inputs for the 1D-TDSE microscopic step.

This module only *generates inputs*: driving-field samples E(t_i) for every
macroscopic point of a synthetic laser focus, per-point box sizes, seeded
random intensities and random probe directions.  It holds none of the
method's arithmetic (no grid, potential, propagator, observable or loss), so
both the HIP path and the CPU oracle can draw identical inputs from it
without sharing any numerical code.

The paper's macroscopic fields come from its infrared propagation code
(section "Infrared Propagation"), which is not reproduced here; the synthetic
Gaussian-beam foci below stand in for them at the paper's scales (focal spots
of tens of micrometres, 1e14 - 2.5e14 W/cm^2, near-infrared drivers, argon).

Units: atomic units for the TDSE (time, field, length), SI-like micrometres /
nanometres for the focus geometry.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Atomic-unit intensity of a field of amplitude 1 a.u. (W/cm^2): I = 3.50945e16 E0^2.
INTENSITY_AU_WCM2 = 3.50945e16
# omega [a.u.] = OMEGA_NM / lambda [nm]  (2 pi c / lambda with c = 137.036 a.u.,
# 1 a.u. of length = 0.0529177 nm).
OMEGA_NM = 45.5634
# Argon ionisation potential used by the configurations (a.u.).
IP_ARGON = 0.5792


def field_amplitude(intensity_wcm2: float) -> float:
    """Peak field (a.u.) of a linearly polarised field of the given intensity."""
    return math.sqrt(intensity_wcm2 / INTENSITY_AU_WCM2)


def omega_from_wavelength(lambda_nm: float) -> float:
    return OMEGA_NM / lambda_nm


def pulse_duration(omega: float, ncycles: float) -> float:
    """Total duration T of an n-cycle sin^2 pulse."""
    return ncycles * 2.0 * math.pi / omega


def n_steps(omega: float, ncycles: float, dt: float) -> int:
    """Number of time steps Nt = ceil(T/dt); the series have Nt+1 samples."""
    return int(math.ceil(pulse_duration(omega, ncycles) / dt - 1e-9))


def sin2_pulse(e0, omega: float, ncycles: float, dt: float, phase=0.0,
               nt: Optional[int] = None, xp=np, i0: int = 0):
    """Samples E_i = e0 sin^2(pi t_i/T) sin(omega t_i + phase), t_i = i dt,
    i = i0..i0+nt, and 0 for t_i > T.  ``e0`` and ``phase`` may be arrays of
    shape [P] (one row per macroscopic point); the result is [P, nt+1] or
    [nt+1].  ``xp`` is numpy or torch (for generation on the device).  A
    window starting at i0 holds bitwise the samples of the full series."""
    T = pulse_duration(omega, ncycles)
    if nt is None:
        nt = n_steps(omega, ncycles, dt) - i0
    if xp is np:
        t = np.arange(i0, i0 + nt + 1, dtype=np.float64) * dt
        e0a = np.asarray(e0, dtype=np.float64)
        pha = np.asarray(phase, dtype=np.float64)
        env = np.where(t <= T, np.sin(np.pi * t / T) ** 2, 0.0)
        if e0a.ndim == 0 and pha.ndim == 0:
            return float(e0a) * env * np.sin(omega * t + float(pha))
        e0a = np.broadcast_to(e0a, np.broadcast(e0a, pha).shape)[:, None]
        pha = np.broadcast_to(pha, e0a.shape[:1])[:, None]
        return e0a * env[None, :] * np.sin(omega * t[None, :] + pha)
    import torch  # generation on a device; plumbing only

    dev = xp["device"] if isinstance(xp, dict) else "cpu"
    t = torch.arange(i0, i0 + nt + 1, dtype=torch.float64, device=dev) * dt
    env = torch.where(t <= T, torch.sin(math.pi * t / T) ** 2, torch.zeros_like(t))
    e0t = torch.as_tensor(e0, dtype=torch.float64, device=dev).reshape(-1, 1)
    pht = torch.as_tensor(phase, dtype=torch.float64, device=dev).reshape(-1, 1)
    return e0t * env[None, :] * torch.sin(omega * t[None, :] + pht)


def gaussian_focus(nr: int, nz: int, w0_um: float, lambda_nm: float, i0_wcm2: float,
                   r_max_w0: float = 1.5, z_max_zr: float = 2.0):
    """Local amplitude and phase of a focused Gaussian beam on an inclusive
    nr x nz grid r in [0, r_max_w0 w0], z in [-z_max_zr z_R, z_max_zr z_R].

      w(z)  = w0 sqrt(1 + (z/z_R)^2),  z_R = pi w0^2 / lambda,  k = 2 pi / lambda
      E0(r,z)  = E0 (w0/w(z)) exp(-r^2/w(z)^2)
      phi(r,z) = atan(z/z_R) + k r^2 z / (2 (z^2 + z_R^2))

    Returns (e0 [nr*nz], phase [nr*nz], r_um [nr*nz], z_um [nr*nz]) with the
    point index p = ir * nz + iz."""
    lam_um = lambda_nm * 1e-3
    zr = math.pi * w0_um ** 2 / lam_um
    k = 2.0 * math.pi / lam_um
    r = np.linspace(0.0, r_max_w0 * w0_um, nr)
    z = np.linspace(-z_max_zr * zr, z_max_zr * zr, nz)
    R, Z = np.meshgrid(r, z, indexing="ij")
    w = w0_um * np.sqrt(1.0 + (Z / zr) ** 2)
    e0 = field_amplitude(i0_wcm2) * (w0_um / w) * np.exp(-(R / w) ** 2)
    phase = np.arctan(Z / zr) + k * R ** 2 * Z / (2.0 * (Z ** 2 + zr ** 2))
    return e0.ravel(), phase.ravel(), R.ravel(), Z.ravel()


def round_up(v: int, m: int) -> int:
    return ((v + m - 1) // m) * m


@dataclass
class Workload:
    """A batch of independent microscopic problems sharing dx, dt and the atom."""
    name: str
    dx: float
    dt: float
    omega: float
    ncycles: float
    nt: int
    n_per: List[int]
    e0: np.ndarray
    phase: np.ndarray
    ip: float = IP_ARGON
    mask_frac: float = 0.1
    mask_pow: float = 0.125
    meta: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return len(self.n_per)

    def point_steps(self) -> int:
        return int(sum(self.n_per)) * self.nt

    def subset(self, rows, name: Optional[str] = None) -> "Workload":
        """The systems `rows` of this batch, in that order, as a batch of their own."""
        rows = [int(r) for r in rows]
        meta = {k: (v[rows] if isinstance(v, np.ndarray) and v.shape[:1] == (self.batch,) else v)
                for k, v in self.meta.items()}
        return Workload(name or f"{self.name}-sub{len(rows)}", self.dx, self.dt, self.omega,
                        self.ncycles, self.nt, [self.n_per[r] for r in rows], self.e0[rows],
                        self.phase[rows], self.ip, self.mask_frac, self.mask_pow, meta)

    def efield(self, rows=None, xp=np, i0: int = 0, nt: Optional[int] = None):
        """Field samples [P, nt+1] (numpy, or torch on a device when xp is
        {"device": dev}); with i0/nt the window of samples i0..i0+nt of the
        full series (nt defaults to the rest of the pulse)."""
        e0, ph = self.e0, self.phase
        if rows is not None:
            e0, ph = e0[rows], ph[rows]
        if nt is None:
            nt = self.nt - i0
        return sin2_pulse(e0, self.omega, self.ncycles, self.dt, ph, nt=nt, xp=xp, i0=i0)


def cfg1_single() -> Workload:
    """Single TDSE: N = 2048, dx = 0.2, dt = 0.05, 800 nm (omega = 0.057),
    10-cycle sin^2, 1.5e14 W/cm^2 (E0 = 0.0654)."""
    om, nc, dt = 0.057, 10, 0.05
    return Workload("single-2048", 0.2, dt, om, nc, n_steps(om, nc, dt), [2048],
                    np.array([field_amplitude(1.5e14)]), np.array([0.0]))


def size_sweep(n: int, batch: int = 1024) -> Workload:
    """Uniform batch of `batch` systems of N = n points with the single-system
    pulse (dx = 0.2, dt = 0.05, 800 nm, 10 cycles, 1.5e14 W/cm^2): the size
    sweep N in {2048, 4096, 8192, 16384}."""
    om, nc, dt = 0.057, 10, 0.05
    return Workload(f"sweep-{batch}x{n}", 0.2, dt, om, nc, n_steps(om, nc, dt), [n] * batch,
                    np.full(batch, field_amplitude(1.5e14)), np.zeros(batch))


def cfg2_focus(nr: int = 32, nz: int = 32) -> Workload:
    """Gaussian focus, 32 r x 32 z points, w0 = 50 um, 800 nm, 2e14 W/cm^2,
    20 cycles, N = 4096, dx = 0.2, dt = 0.05."""
    om, nc, dt = 0.057, 20, 0.05
    e0, ph, r, z = gaussian_focus(nr, nz, 50.0, 800.0, 2e14)
    return Workload(f"focus-{nr}x{nz}-4096", 0.2, dt, om, nc, n_steps(om, nc, dt),
                    [4096] * (nr * nz), e0, ph, meta={"r_um": r, "z_um": z})


def cfg3_uneven(batch: int = 4096, wide: bool = False, seed: int = 250704115) -> Workload:
    """Uneven batch: intensities log-uniform in [5e13, 4e14] W/cm^2, 1300 nm
    (omega = 0.0351), 12-cycle sin^2, dt = 0.025, dx = 0.2.  Box half-width
    3 E0/omega^2 + 50 a.u., N = clamp(roundup_256(2 h / dx), 2048, 16384).
    ``wide``: N drawn log-uniform in [2048, 16384] (rounded to 256) with the
    same intensities, to span the stated size range."""
    om, nc, dt, dx = 0.0351, 12, 0.025, 0.2
    rng = np.random.default_rng(seed)
    inten = np.exp(rng.uniform(math.log(5e13), math.log(4e14), size=batch))
    e0 = np.sqrt(inten / INTENSITY_AU_WCM2)
    if wide:
        nlog = rng.uniform(math.log(2048), math.log(16384), size=batch)
        n_per = [min(16384, max(2048, round_up(int(math.exp(v)), 256))) for v in nlog]
    else:
        h = 3.0 * e0 / om ** 2 + 50.0
        n_per = [min(16384, max(2048, round_up(int(math.ceil(2 * hv / dx)), 256))) for hv in h]
    phase = np.zeros(batch)
    return Workload(("uneven-wide" if wide else "uneven") + f"-{batch}", dx, dt, om, nc,
                    n_steps(om, nc, dt), n_per, e0, phase)


def cfg4_adjoint(batch: int = 256, seed: int = 250704116) -> Workload:
    """Adjoint batch: 256 systems, N = 4096, dx = 0.2, dt = 0.05, 800 nm
    10-cycle pulses, E0 uniform in [0.05, 0.075]; loss band H21-H31."""
    om, nc, dt = 0.057, 10, 0.05
    rng = np.random.default_rng(seed)
    e0 = rng.uniform(0.05, 0.075, size=batch)
    return Workload(f"adjoint-{batch}-4096", 0.2, dt, om, nc, n_steps(om, nc, dt),
                    [4096] * batch, e0, np.zeros(batch), meta={"band": (21, 31)})


def cfg5_volume(nr: int = 64, nz: int = 256) -> Workload:
    """Full focal volume: 64 r x 256 z, w0 = 80 um, 1030 nm, 2.5e14 W/cm^2,
    30 cycles, N = 8192, dx = 0.15, dt = 0.02."""
    om, nc, dt = omega_from_wavelength(1030.0), 30, 0.02
    e0, ph, r, z = gaussian_focus(nr, nz, 80.0, 1030.0, 2.5e14)
    return Workload(f"volume-{nr}x{nz}-8192", 0.15, dt, om, nc, n_steps(om, nc, dt),
                    [8192] * (nr * nz), e0, ph, meta={"r_um": r, "z_um": z, "band": (25, 35)})


def cfg5_axis(nz: int = 256) -> Workload:
    """The on-axis (r = 0) points of the full focal volume: the systems whose
    yields make up the volume's adjoint loss (the other rows get an all-zero
    accel_bar and no reverse sweep)."""
    w = cfg5_volume(64, nz)
    keep = np.nonzero(w.meta["r_um"] == 0.0)[0]
    return Workload(f"volume-axis-{len(keep)}-8192", w.dx, w.dt, w.omega, w.ncycles, w.nt,
                    [w.n_per[i] for i in keep], w.e0[keep], w.phase[keep],
                    meta={"r_um": w.meta["r_um"][keep], "z_um": w.meta["z_um"][keep],
                          "band": (25, 35)})


def probe_directions(shape, d: int, seed0: int = 250704117) -> np.ndarray:
    """Seeded N(0,1) direction number d for finite-difference checks."""
    return np.random.default_rng(seed0 + d).standard_normal(shape)


def random_state(n: int, seed: int, width: float = 10.0, k0: float = 0.0,
                 dx: float = 0.2) -> np.ndarray:
    """A seeded smooth complex initial state (Gaussian envelope times a random
    low-order complex polynomial), used where a non-eigenstate start is
    wanted.  Not normalised."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) - 0.5 * (n - 1)) * dx
    c = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    poly = c[0] + c[1] * (x / width) + c[2] * (x / width) ** 2 + c[3] * (x / width) ** 3
    return np.exp(-(x / width) ** 2 + 1j * k0 * x) * poly
