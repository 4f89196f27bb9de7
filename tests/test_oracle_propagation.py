"""Pins of the oracle's forward propagation against things other than itself:
dense textbook propagators, the exact discrete spectral solution, continuum
closed forms, conservation laws and Ehrenfest's theorem."""
import numpy as np
import pytest
from scipy.fft import dst

import oracle
import tdse_inputs as ti
from dense_reference import cayley, dense_h, exact_step, grid_x

A_AR = 1.1891671  # soft-core a giving Ip = 0.5792 at dx = 0.2 (pinned in test_oracle_ground_state)


def test_one_step_equals_dense_cayley_times_phase():
    """One oracle step = diag(exp(-i dt E x)) (I + i dt/2 H)^-1 (I - i dt/2 H)
    with the dense symmetric H = M2^-1(-D2/2) + V (Sec. 1D-TSDE
    Implementation, CN substeps)."""
    rng = np.random.default_rng(1)
    for n, dx, dt, a, e in [(64, 0.3, 0.05, 1.2, 0.07), (97, 0.2, 0.1, 0.8, -0.3)]:
        h, x = dense_h(n, dx, a)
        psi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        ref = np.exp(-1j * dt * e * x) * (cayley(h, dt) @ psi)
        out = oracle.step(psi, dx, dt, a, 1.0, e)
        assert np.max(np.abs(out - ref)) / np.max(np.abs(ref)) < 1e-14


def test_free_propagation_equals_exact_dst_solution():
    """Free particle, no field, no absorber: M2 and D2 are both diagonalised by
    the orthonormal DST-I, so psi(n dt) = S diag(g_k^n) S psi0 with
    g_k = (1 - i dt T_k/2)/(1 + i dt T_k/2), T_k = -lam_k/(2 mu_k)."""
    n, dx, dt, steps = 256, 0.25, 0.05, 400
    x = grid_x(n, dx)
    psi0 = np.exp(-(x - 3.0) ** 2 / 8.0 + 1.2j * x)
    k = np.arange(1, n + 1)
    lam = (2.0 * np.cos(k * np.pi / (n + 1)) - 2.0) / dx ** 2
    mu = 1.0 + dx ** 2 * lam / 12.0
    tk = -lam / (2.0 * mu)
    g = (1 - 0.5j * dt * tk) / (1 + 0.5j * dt * tk)
    coef = dst(psi0, type=1, norm="ortho")
    ref = dst(coef * g ** steps, type=1, norm="ortho")
    out = oracle.propagate(np.zeros(steps + 1), psi0, dx, dt, 1.0, z=0.0, mask_frac=0.0,
                           want_psi=True)
    assert np.max(np.abs(out["psi_final"] - ref)) < 1e-12 * np.max(np.abs(psi0))


@pytest.mark.parametrize("dx,dt", [(0.2, 0.02), (0.1, 0.01)])
def test_free_gaussian_matches_continuum_closed_form(dx, dt):
    """Spreading and drift of a free Gaussian: sigma(t)^2 = s0^2 + t^2/(4 s0^2),
    <x>(t) = x0 + k0 t (hbar = m = 1); the discretisation error is small and
    shrinks with dx, dt."""
    s0, x0, k0, t_end = 1.5, -5.0, 0.6, 10.0
    n = int(round(120.0 / dx)) | 1
    x = grid_x(n, dx)
    psi0 = (2 * np.pi * s0 ** 2) ** -0.25 * np.exp(-(x - x0) ** 2 / (4 * s0 ** 2) + 1j * k0 * x)
    steps = int(round(t_end / dt))
    out = oracle.propagate(np.zeros(steps + 1), psi0, dx, dt, 1.0, z=0.0, mask_frac=0.0,
                           want_psi=True)
    p = np.abs(out["psi_final"]) ** 2 * dx
    mean = np.sum(x * p)
    var = np.sum((x - mean) ** 2 * p)
    sig_ref = np.sqrt(s0 ** 2 + t_end ** 2 / (4 * s0 ** 2))
    tol = 2e-4 if dx == 0.2 else 6e-5
    assert abs(mean - (x0 + k0 * t_end)) < tol
    assert abs(np.sqrt(var) - sig_ref) / sig_ref < tol
    assert abs(out["norm"][-1] - 1.0) < 1e-12


def test_constant_field_accelerates_electron_against_field():
    """Free particle in a constant field e: H = p^2/2 + x e, so
    d^2<x>/dt^2 = -e exactly; the split step converges to it (first order)."""
    e, s0 = 0.02, 2.0
    errs = []
    for dt in (0.1, 0.05):
        n, dx = 801, 0.2
        x = grid_x(n, dx)
        psi0 = (2 * np.pi * s0 ** 2) ** -0.25 * np.exp(-x ** 2 / (4 * s0 ** 2))
        steps = int(round(20.0 / dt))
        out = oracle.propagate(np.full(steps + 1, e), psi0, dx, dt, 1.0, z=0.0, mask_frac=0.0)
        t = np.arange(steps + 1) * dt
        errs.append(np.max(np.abs(out["xexp"] - (-0.5 * e * t ** 2))))
    assert errs[1] < 0.2 * 0.5 * e * 20.0 ** 2 * 0.05  # close to -e t^2/2, not +e t^2/2
    assert errs[1] < 0.7 * errs[0]                         # converging as dt shrinks


def test_norm_conserved_without_absorber_single_2048():
    """The scheme is the Cayley transform of a real symmetric H, hence unitary:
    over the 22 047 steps of the single-system workload the norm stays 1 to
    1e-12 when the absorber is off."""
    w = ti.cfg1_single()
    psi0, _, _ = oracle.ground_state(2048, 0.2, A_AR)
    out = oracle.propagate(w.efield()[0], psi0, 0.2, w.dt, A_AR, mask_frac=0.0)
    assert np.max(np.abs(out["norm"] - 1.0)) < 1e-12


def _ehrenfest_residuals(dt, pair_previous):
    n, dx, a = 2048, 0.2, A_AR
    psi0, _, _ = oracle.ground_state(n, dx, a)
    om, nc = 0.057, 2
    nt = ti.n_steps(om, nc, dt)
    e = ti.sin2_pulse(0.04, om, nc, dt, nt=nt)
    out = oracle.propagate(e, psi0, dx, dt, a, mask_frac=0.0, want_psi=True)
    assert np.sum(np.abs(out["psi_final"][:100]) ** 2) < 1e-10   # edges stay empty
    X, acc, nrm = out["xexp"], out["accel"], out["norm"]
    xdd = (X[2:] - 2 * X[1:-1] + X[:-2]) / dt ** 2
    dv_mean = acc[1:-1] - e[1:-1] * nrm[1:-1]      # <dV/dx> at sample i
    kick = e[:-2] if pair_previous else e[1:-1]
    res = xdd + dv_mean + kick * nrm[1:-1]
    return np.linalg.norm(res) / np.linalg.norm(xdd)


@pytest.mark.slow
def test_ehrenfest_theorem():
    """d^2<x>/dt^2 = -<dV/dx> - E (Ehrenfest, appendix "Microscopic source
    terms").  With the field kick of step i-1 -> i paired to sample i the
    residual is small and shrinks quickly with dt; the literal E_i pairing
    converges at first order (the split step)."""
    r1 = _ehrenfest_residuals(0.05, True)
    r2 = _ehrenfest_residuals(0.025, True)
    assert r1 < 2e-3
    assert r2 < r1 / 2.5
    l1 = _ehrenfest_residuals(0.05, False)
    l2 = _ehrenfest_residuals(0.025, False)
    assert 1.6 < l1 / l2 < 2.4


def test_split_step_orders_against_expm():
    """64-point grid vs scipy expm: without field the scheme is second order;
    with a field the Lie splitting makes it first order."""
    n, dx, a = 64, 0.5, 1.2
    h, x = dense_h(n, dx, a)
    evals, evecs = np.linalg.eigh(h)
    psi0 = (evecs[:, 0] + 0.3 * evecs[:, 2] + 0.2j * evecs[:, 5]).astype(complex)
    T = 1.0

    def err(dt, e):
        steps = int(round(T / dt))
        out = oracle.propagate(np.full(steps + 1, e), psi0, dx, dt, a, mask_frac=0.0,
                               want_psi=True)
        ref = exact_step(h, x, T, e) @ psi0
        return np.linalg.norm(out["psi_final"] - ref)

    e0 = [err(dt, 0.0) for dt in (0.1, 0.05, 0.025)]
    e1 = [err(dt, 0.3) for dt in (0.1, 0.05, 0.025)]
    for r in (e0[0] / e0[1], e0[1] / e0[2]):
        assert 3.6 < r < 4.4
    for r in (e1[0] / e1[1], e1[1] / e1[2]):
        assert 1.7 < r < 2.3


def test_absorber_profile_and_absorption():
    """Mask with fraction 0.1: 1 for |x| <= 0.8 x_max (a tenth of the whole
    grid absorbs at each side), below 1 and strictly decreasing beyond it,
    0 at the two outermost points; a packet sent into it is absorbed, not
    reflected."""
    n, dx = 601, 0.2
    m = oracle.mask(n, dx, 0.1, 0.125)
    x = grid_x(n, dx)
    xmax = x[-1]
    inner = np.abs(x) <= 0.8 * xmax
    assert np.all(m[inner] == 1.0)
    assert np.all(m[~inner] < 1.0)
    assert np.sum(~inner) == 2 * 60          # 10 % of the 600 intervals at each side
    assert m[0] == 0.0 and m[-1] == 0.0
    right = m[x > 0.8 * xmax]
    assert np.all(np.diff(right) < 0)
    psi0 = np.exp(-(x - 30.0) ** 2 / 8.0 + 2.0j * x)
    psi0 /= np.sqrt(dx * np.sum(np.abs(psi0) ** 2))
    out = oracle.propagate(np.zeros(1001), psi0, dx, 0.05, 1.0, z=0.0, mask_frac=0.1,
                           want_psi=True)
    assert out["norm"][-1] < 0.05
    assert np.all(np.diff(out["norm"]) <= 4e-15)          # the mask only removes norm
    assert dx * np.sum(np.abs(out["psi_final"][x < 0]) ** 2) < 0.01


@pytest.mark.parametrize("power", [0.125, 0.5, 1.0])
@pytest.mark.parametrize("frac", [0.1, 0.25])
def test_absorber_exponent_at_exact_cosine_points(frac, power):
    """Values of the cos^p profile where the cosine is exact: with
    u = (|x| - x_a)/(x_max - x_a), u = 1/3, 1/2, 2/3 give cos = sqrt(3)/2,
    2^-1/2, 1/2, so m = (sqrt(3)/2)^p, 2^(-p/2), 2^-p (for p = 1/8:
    2^(-1/16) at u = 1/2 and 2^(-1/8) at u = 2/3).  The grid has 2M
    intervals with M a multiple of 30, so these u fall on grid points; a
    wrong exponent, a wrong x_a or a wrong fraction fails here."""
    big_m = 60
    n, dx = 2 * big_m + 1, 0.3
    m = oracle.mask(n, dx, frac, power)
    # x_j = (j - M) dx, x_max = M dx, x_a = (1 - 2 frac) M dx: u = 1/3 at
    # |j - M| = M (1 - 2 frac + 2 frac / 3), and so on
    for u, ref in [(1.0 / 3.0, (np.sqrt(3.0) / 2.0) ** power), (0.5, 2.0 ** (-0.5 * power)),
                   (2.0 / 3.0, 2.0 ** (-power))]:
        d = big_m * (1.0 - 2.0 * frac + 2.0 * frac * u)
        assert abs(d - round(d)) < 1e-9
        for j in (big_m + int(round(d)), big_m - int(round(d))):
            assert abs(m[j] - ref) < 4e-15, (u, j, m[j], ref)
    # the first point past x_a is the first one below 1
    k_a = big_m * (1.0 - 2.0 * frac)
    assert m[big_m + int(round(k_a))] == 1.0 and m[big_m + int(round(k_a)) + 1] < 1.0


def test_propagate_batch_equals_single_propagations():
    """The threaded batch oracle gives, bitwise, what one ragged system at a
    time gives: rows of different sizes and fields, their initial states
    read at non-contiguous offsets of one buffer (gaps between them), four
    host threads."""
    import ctypes

    rng = np.random.default_rng(11)
    ns = [64, 97, 33, 128, 64]
    nt, dx, dt, a = 40, 0.3, 0.05, 1.1
    efield = rng.uniform(-0.1, 0.1, size=(len(ns), nt + 1))
    psis = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in ns]
    off = np.zeros(len(ns) + 1, np.int64)
    gap = 5
    for b, n in enumerate(ns):
        off[b + 1] = off[b] + n + gap
    buf = np.full(int(off[-1]), np.nan + 1j * np.nan)
    for b, n in enumerate(ns):
        buf[off[b]:off[b] + n] = psis[b]
    acc = np.empty((len(ns), nt + 1))
    xe = np.empty_like(acc)
    nr = np.empty_like(acc)
    lib = oracle._load()
    n_per = np.array(ns, np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.tdse_ref_propagate_batch(len(ns), n_per.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), dx, dt, a,
                                 1.0, 0.1, 0.125, nt, efield.ctypes.data_as(dp),
                                 buf.ctypes.data_as(dp), acc.ctypes.data_as(dp),
                                 xe.ctypes.data_as(dp), nr.ctypes.data_as(dp), 4)
    assert st == 0
    for b in range(len(ns)):
        ref = oracle.propagate(efield[b], psis[b], dx, dt, a, mask_frac=0.1)
        assert np.array_equal(acc[b], ref["accel"])
        assert np.array_equal(xe[b], ref["xexp"])
        assert np.array_equal(nr[b], ref["norm"])
    # the wrapper with its contiguous offsets gives the same rows
    out = oracle.propagate_batch(efield, psis, dx, dt, a, mask_frac=0.1, nthreads=3)
    assert np.array_equal(out["accel"], acc)
