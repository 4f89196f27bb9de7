"""Pins of the oracle's harmonic-yield loss and discrete adjoint: numpy FFT
bins, Parseval, finite differences, and reverse-mode autograd of an
independent dense formulation of the forward map."""
import numpy as np
import pytest
import torch

import oracle
import tdse_inputs as ti
from dense_reference import cayley, dense_h, grid_x


def _series(ntp1, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(ntp1) * 0.05
    return (np.sin(0.057 * 23 * t) * np.exp(-((t - t[-1] / 2) / 300) ** 2)
            + 0.01 * rng.standard_normal(ntp1))[None, :]


def test_band_dft_equals_numpy_fft_bins():
    ntp1, dt, om = 4001, 0.05, 0.057
    a = _series(ntp1, 0)
    loss, _ = oracle.harmonic_yield(a, dt, om, 21, 31)
    nt = ntp1 - 1
    w = np.sin(np.pi * np.arange(ntp1) / nt) ** 2
    X = np.fft.fft(w * a[0])
    kb = oracle.band_bins(ntp1, dt, om, 21, 31)
    dw = 2 * np.pi / (ntp1 * dt)
    assert len(kb) > 10
    assert abs(loss[0] - dw * np.sum(np.abs(dt * X[kb]) ** 2)) < 1e-13 * loss[0]


def test_parseval_over_all_bins():
    """With the band covering every one-sided bin, the yield obeys Parseval:
    sum_k c_k |A_k|^2 = dt^2 (nt+1) sum_i (w_i a_i)^2 (c_0 = 1, c_k = 2)."""
    ntp1, dt = 1001, 0.05
    a = _series(ntp1, 1)
    om = 1.0
    kb = oracle.band_bins(ntp1, dt, om, 0.0, 1e9)
    assert len(kb) == ntp1 // 2 + 1
    loss, _ = oracle.harmonic_yield(a, dt, om, 0.0, 1e9)
    _, _ = loss, None
    nt = ntp1 - 1
    w = np.sin(np.pi * np.arange(ntp1) / nt) ** 2
    dw = 2 * np.pi / (ntp1 * dt)
    # loss counts each one-sided bin once; add the mirrored bins (all but k = 0)
    amp0 = dt * np.sum(w * a[0])
    two_sided = 2 * loss[0] / dw - abs(amp0) ** 2
    assert abs(two_sided - dt ** 2 * ntp1 * np.sum((w * a[0]) ** 2)) < 1e-12 * two_sided


def test_yield_gradient_matches_central_differences():
    ntp1, dt, om = 801, 0.05, 0.3
    a = _series(ntp1, 2)
    loss, abar = oracle.harmonic_yield(a, dt, om, 3, 7)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(a.shape)
        h = 1e-4
        lp, _ = oracle.harmonic_yield(a + h * v, dt, om, 3, 7)
        lm, _ = oracle.harmonic_yield(a - h * v, dt, om, 3, 7)
        fd = (lp[0] - lm[0]) / (2 * h)
        assert abs(fd - np.sum(abar * v)) < 1e-9 * abs(fd)


# ---------------------------------------------------------------- adjoint

def _toy(n=128, dx=0.4, a=1.1, om=0.25, nc=3, dt=0.05, e0=0.12):
    nt = ti.n_steps(om, nc, dt)
    e = ti.sin2_pulse(e0, om, nc, dt, nt=nt)
    psi0, _, _ = oracle.ground_state(n, dx, a)
    return dict(n=n, dx=dx, a=a, om=om, dt=dt, nt=nt, e=e, psi0=psi0)


def _loss(c, e):
    out = oracle.propagate(e, c["psi0"], c["dx"], c["dt"], c["a"], mask_frac=0.2)
    l, abar = oracle.harmonic_yield(out["accel"][None, :], c["dt"], c["om"], 3, 9)
    return l[0], abar[0]


def test_adjoint_matches_central_differences_with_absorber():
    c = _toy()
    _, abar = _loss(c, c["e"])
    g, _ = oracle.adjoint(c["e"], c["psi0"], abar, c["dx"], c["dt"], c["a"], mask_frac=0.2,
                          k=64)
    for d in range(4):
        v = ti.probe_directions(c["e"].shape, d)
        h = 1e-6
        lp, _ = _loss(c, c["e"] + h * v)
        lm, _ = _loss(c, c["e"] - h * v)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ v) < 1e-6 * abs(fd)


def test_adjoint_independent_of_checkpoint_interval():
    c = _toy(n=96, nc=2)
    _, abar = _loss(c, c["e"])
    gs = [oracle.adjoint(c["e"], c["psi0"], abar, c["dx"], c["dt"], c["a"], mask_frac=0.2,
                         k=k)[0] for k in (1, 16, 256, c["nt"] + 5)]
    for g in gs[1:]:
        assert np.array_equal(g, gs[0])


def test_adjoint_equals_autograd_of_dense_forward():
    """Reverse-mode autograd (torch, complex128) of an independent dense
    formulation psi^{i+1} = m * exp(-i dt E_i x) * Cayley(H) psi^i with the
    symmetric dense H gives the same gradient as the oracle's adjoint."""
    n, dx, a, dt, nt = 40, 0.5, 1.0, 0.1, 60
    h, x = dense_h(n, dx, a)
    u = torch.tensor(cayley(h, dt))
    xs = torch.tensor(x)
    dv = torch.tensor(x * (x ** 2 + a ** 2) ** -1.5)
    m = torch.tensor(oracle.mask(n, dx, 0.25, 0.125))
    rng = np.random.default_rng(5)
    e_np = 0.3 * rng.standard_normal(nt + 1)
    abar_np = rng.standard_normal(nt + 1)
    psi0 = ti.random_state(n, 7, width=4.0, dx=dx)
    e = torch.tensor(e_np, requires_grad=True)
    psi = torch.tensor(psi0)
    accel = []
    for i in range(nt + 1):
        p = psi.real ** 2 + psi.imag ** 2
        accel.append(dx * torch.sum(p * (dv + e[i])))
        if i < nt:
            psi = m * torch.exp(-1j * dt * e[i] * xs) * (u @ psi)
    accel = torch.stack(accel)
    (accel * torch.tensor(abar_np)).sum().backward()
    g_ref = e.grad.numpy()
    g, acc = oracle.adjoint(e_np, psi0, abar_np, dx, dt, a, mask_frac=0.25, k=7)
    assert np.max(np.abs(acc - accel.detach().numpy())) < 1e-12 * np.max(np.abs(acc))
    assert np.max(np.abs(g - g_ref)) < 1e-11 * np.max(np.abs(g_ref))


@pytest.mark.slow
def test_adjoint_fd_on_adjoint_workload_system():
    """One system of the adjoint workload (N = 4096, 800 nm, 10 cycles,
    H21-H31 band): gradient vs central differences along seeded directions."""
    w = ti.cfg4_adjoint(batch=1)
    a_sc = 1.1891671
    psi0, _, _ = oracle.ground_state(4096, 0.2, a_sc)
    e = w.efield()[0]

    def loss(ef):
        out = oracle.propagate(ef, psi0, 0.2, w.dt, a_sc, mask_frac=0.1)
        l, ab = oracle.harmonic_yield(out["accel"][None, :], w.dt, w.omega, 21, 31)
        return l[0], ab[0]

    l0, abar = loss(e)
    g, _ = oracle.adjoint(e, psi0, abar, 0.2, w.dt, a_sc, mask_frac=0.1, k=256)
    v = ti.probe_directions(e.shape, 0)
    h = 1e-6
    fd = (loss(e + h * v)[0] - loss(e - h * v)[0]) / (2 * h)
    assert abs(fd - g @ v) < 1e-5 * abs(fd)
