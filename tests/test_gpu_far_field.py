"""GPU parity of the far-field path (band spectrum, its adjoint, the
far-field diffraction sum and its adjoint) against the oracle, and the
gradient of an on-axis far-field yield through the whole chain (field
samples -> TDSE -> band spectrum -> far field) against central differences
of the GPU forward map."""
import numpy as np
import pytest

import oracle
import tdse_inputs as ti

pytestmark = pytest.mark.gpu

AU_TIME_S = 2.4188843265857e-17
C_LIGHT = 299792458.0


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def test_band_spectrum_and_adjoint_match_oracle(lib, torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(11)
    nt, dt, om = 700, 0.05, 0.25
    a = rng.standard_normal((5, nt + 1))
    kb, A = oracle.band_amplitudes(a, dt, om, 3, 9)
    k_lo, nk = lib.tdse_harmonic_band(nt, dt, om, 3, 9)
    assert k_lo == kb[0] and nk == len(kb)
    amp = torch.empty(5, nk, dtype=torch.complex128, device=dev)
    lib.tdse_band_dft(5, nt, dt, om, 3, 9, torch.tensor(a, device=dev), amp)
    torch.cuda.synchronize()
    assert rel(amp.cpu().numpy(), A) < 1e-12
    G = rng.standard_normal((5, nk)) + 1j * rng.standard_normal((5, nk))
    abar = torch.empty(5, nt + 1, dtype=torch.float64, device=dev)
    lib.tdse_band_dft_adjoint(5, nt, dt, om, 3, 9, torch.tensor(G, device=dev), abar)
    torch.cuda.synchronize()
    assert rel(abar.cpu().numpy(), oracle.band_adjoint(G, nt + 1, dt, kb)) < 1e-12


def _geometry(rng, n_rho, n_z, nk, n_obs):
    rho = np.linspace(0.0, 60e-6, n_rho)
    z = np.linspace(-2e-3, 2e-3, n_z)
    w = rng.uniform(0.5, 1.5, n_rho * n_z) * 1e-12
    kw = np.linspace(2.0e8, 3.0e8, nk)                    # 1/m, XUV
    ro = np.linspace(0.0, 2e-3, n_obs)
    return rho, z, w, kw, ro, 0.5


@pytest.mark.parametrize("n_rho,n_z,nk,n_obs", [(6, 9, 5, 11), (1, 1, 1, 1), (17, 33, 3, 8)])
def test_far_field_and_adjoint_match_oracle(lib, torch_dev, n_rho, n_z, nk, n_obs):
    torch, dev = torch_dev
    rng = np.random.default_rng(n_rho * 100 + n_z)
    rho, z, w, kw, ro, zo = _geometry(rng, n_rho, n_z, nk, n_obs)
    P = n_rho * n_z
    S = rng.standard_normal((P, nk)) + 1j * rng.standard_normal((P, nk))
    t = lambda x: torch.tensor(np.ascontiguousarray(x), device=dev)
    print(f"far field n_rho={n_rho} n_z={n_z} nk={nk} n_obs={n_obs}", flush=True)
    E = torch.empty(n_obs, nk, dtype=torch.complex128, device=dev)
    lib.tdse_far_field(t(rho), t(z), t(w), t(kw), t(S), t(ro), zo, E)
    Eb = rng.standard_normal((n_obs, nk)) + 1j * rng.standard_normal((n_obs, nk))
    Sb = torch.empty(P, nk, dtype=torch.complex128, device=dev)
    lib.tdse_far_field(t(rho), t(z), t(w), t(kw), t(Eb), t(ro), zo, Sb, adjoint=True)
    torch.cuda.synchronize()
    assert rel(E.cpu().numpy(), oracle.far_field(S, rho, z, w, kw, ro, zo)) < 1e-10
    assert rel(Sb.cpu().numpy(), oracle.far_field_adjoint(Eb, rho, z, w, kw, ro, zo)) < 1e-10


def test_on_axis_far_field_yield_gradient(lib, torch_dev):
    """l = sum over the band of |E(rho = 0, omega)|^2 for a 2 r x 3 z focus;
    dl/dE(t) through TDSEFunction, BandSpectrum and FarField against central
    differences of the GPU forward map (bar 1e-5)."""
    torch, dev = torch_dev
    from paper_2507_04115_amd import autograd as AG

    om, nc, dt, dx, a = 0.25, 3, 0.05, 0.4, 1.1
    nt = ti.n_steps(om, nc, dt)
    nr, nz = 2, 3
    e0, ph, r_um, z_um = ti.gaussian_focus(nr, nz, 50.0, 800.0, 2e14)
    efield = ti.sin2_pulse(e0, om, nc, dt, phase=ph, nt=nt)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    batch = AG.TDSEBatch(p, [256] * (nr * nz), adjoint_k=64, store_checkpoints=True)
    k_lo, nk = lib.tdse_harmonic_band(nt, dt, om, 3, 9)
    omega_si = 2 * np.pi * (k_lo + np.arange(nk)) / ((nt + 1) * dt) / AU_TIME_S
    rho = np.unique(r_um) * 1e-6
    z = np.unique(z_um) * 1e-6
    drho = rho[1] - rho[0]
    dz = z[1] - z[0]
    w = np.outer(rho * drho, np.full(nz, dz)).ravel()
    w[:nz] = 0.25 * drho ** 2 * dz            # the axis cell: int_0^{drho/2} rho drho
    geom = AG.FarFieldGeometry(rho, z, w, omega_si / C_LIGHT, [0.0, 1e-4], 0.5, device=dev)

    def loss(E):
        amp = AG.BandSpectrum.apply(batch(E), dt, om, 3, 9)
        field = AG.FarField.apply(amp, geom)
        return (field[0].abs() ** 2).sum()

    E = torch.tensor(efield, dtype=torch.float64, device=dev, requires_grad=True)
    l0 = loss(E)
    l0.backward()
    g = E.grad.detach()
    assert torch.count_nonzero(g) > 0
    h = 1e-6
    for d in range(2):
        v = torch.tensor(ti.probe_directions(E.shape, d), dtype=torch.float64, device=dev)
        with torch.no_grad():
            fd = float((loss(E + h * v) - loss(E - h * v)) / (2 * h))
        ad = float((g * v).sum())
        print(f"  direction {d}: FD {fd:.10e} adjoint {ad:.10e}", flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(fd)
    batch.close()
