"""Spectral-phase driver parametrisation (paper_2507_04115_amd.driver) on the
CPU: identity at c = 0, a constant phase is a plain spectral rotation, the
band covers the pulse's spectrum, and autograd through the FFT map agrees
with central differences."""
import math

import numpy as np
import pytest
import torch

import tdse_inputs as ti
from paper_2507_04115_amd.driver import SpectralPhase


@pytest.fixture(scope="module")
def field():
    om, nc, dt = 0.25, 3, 0.05
    nt = ti.n_steps(om, nc, dt)
    e0, ph, _, _ = ti.gaussian_focus(2, 3, 50.0, 800.0, 2e14)
    E = ti.sin2_pulse(e0, om, nc, dt, phase=ph, nt=nt)
    return torch.tensor(E, dtype=torch.float64), om, dt


def test_zero_phase_is_identity(field):
    E, _, _ = field
    sp = SpectralPhase(E, 64)
    assert torch.allclose(sp(torch.zeros(64, dtype=torch.float64)), E, rtol=0, atol=1e-15)


def test_band_covers_the_carrier(field):
    E, om, dt = field
    sp = SpectralPhase(E, 64)
    k_carrier = om * E.shape[1] * dt / (2 * math.pi)
    assert sp.band[0] < k_carrier < sp.band[1]


def test_constant_phase_rotates_the_analytic_signal(field):
    """A constant phase theta on every positive-frequency bin (DC and Nyquist
    carry no spectrum here) maps E to cos(theta) E - sin(theta) H[E]."""
    E, _, _ = field
    sp = SpectralPhase(E, 8, threshold=0.0)   # band = every bin
    th = 0.7
    Ec = sp(torch.full((8,), th, dtype=torch.float64))
    spec = torch.fft.rfft(E, dim=1)
    hil = torch.fft.irfft(-1j * spec, n=E.shape[1], dim=1)   # Hilbert transform
    ref = math.cos(th) * E - math.sin(th) * hil
    assert torch.allclose(Ec, ref, rtol=0, atol=1e-12 * float(E.abs().max()))


def test_gradient_matches_central_differences(field):
    E, _, _ = field
    sp = SpectralPhase(E, 16)
    w = torch.tensor(ti.probe_directions(E.shape, 0), dtype=torch.float64)
    c = torch.tensor(np.random.default_rng(3).normal(0.0, 0.5, 16), dtype=torch.float64,
                     requires_grad=True)
    loss = lambda cc: ((sp(cc) * w).sum() ** 2)
    loss(c).backward()
    h = 1e-6
    for d in range(3):
        v = torch.tensor(np.random.default_rng(10 + d).standard_normal(16), dtype=torch.float64)
        with torch.no_grad():
            fd = float((loss(c + h * v) - loss(c - h * v)) / (2 * h))
        ad = float((c.grad * v).sum())
        assert abs(fd - ad) <= 1e-7 * abs(fd)
