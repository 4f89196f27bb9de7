"""Pin of the oracle's Gabor transform against the closed form of a windowed
cosine: for a(t) = cos(W t) and a window well inside the record,
dt sum_i a_i exp(-(t_i-t_c)^2/(2 s^2)) exp(-i w t_i)
= s sqrt(pi/2) [exp(-s^2 (w-W)^2/2 - i (w-W) t_c) + exp(-s^2 (w+W)^2/2 - i (w+W) t_c)]
up to aliasing terms of order exp(-s^2 (2 pi/dt - w - W)^2 / 2) (Poisson
summation), far below rounding here."""
import numpy as np

import oracle


def test_windowed_cosine_closed_form():
    dt, nt, W, s = 0.05, 8000, 1.3, 12.0
    t = dt * np.arange(nt + 1)
    a = np.cos(W * t)
    tc = np.array([120.0, 200.0, 260.0])
    w = np.linspace(0.5, 2.5, 41)
    G = oracle.gabor(a, dt, tc, w, s)[0]
    for c, t0 in enumerate(tc):
        amp = s * np.sqrt(np.pi / 2) * (np.exp(-s ** 2 * (w - W) ** 2 / 2 - 1j * (w - W) * t0)
                                          + np.exp(-s ** 2 * (w + W) ** 2 / 2 - 1j * (w + W) * t0))
        ref = np.abs(amp) ** 2
        assert np.max(np.abs(G[c] - ref)) < 1e-9 * np.max(ref)
