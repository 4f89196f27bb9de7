"""Pins of the oracle's Fourier zero-padding resampler: band-limited periodic
signals are reproduced exactly between the coarse samples (closed form), and
the coarse samples themselves are reproduced at the coincident fine points."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("M,r", [(64, 4), (75, 3), (128, 10)])
def test_band_limited_signal_is_reproduced(M, r):
    dtc = 0.7
    T = M * dtc
    dt = dtc / r
    rng = np.random.default_rng(M)
    freqs = rng.choice(np.arange(1, (M - 1) // 2), 5, replace=False) / T
    amps = rng.uniform(0.2, 1.0, 5)
    phs = rng.uniform(0, 2 * np.pi, 5)
    f = lambda t: 0.3 + sum(a * np.cos(2 * np.pi * q * t + p) for a, q, p in zip(amps, freqs, phs))
    coarse = f(dtc * np.arange(M))
    nt = M * r - 1
    fine = oracle.resample_field(coarse, dtc, dt, nt)[0]
    assert np.max(np.abs(fine - f(dt * np.arange(nt + 1)))) < 1e-12


def test_coarse_samples_are_kept():
    M, r = 90, 5
    x = np.random.default_rng(9).standard_normal((3, M))
    fine = oracle.resample_field(x, 0.1, 0.1 / r, M * r - 1)
    assert np.max(np.abs(fine[:, ::r] - x)) < 1e-12
