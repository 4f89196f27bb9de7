"""GPU parity of the electron energy distribution (tdse_plan_energy_spectrum)
against the oracle: a ragged batch of random states, the Lorentzian of an
eigenstate, and a workspace that holds only one wavefront of solves (each lane
then takes many (system, energy) items)."""
import numpy as np
import pytest

import oracle
import oracle_side
import tdse_inputs as ti

pytestmark = pytest.mark.gpu

A = 1.1891671


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _c2d(psi):
    return np.ascontiguousarray(np.asarray(psi, np.complex128)).view(np.float64)


@pytest.mark.parametrize("lanes", [None, 64])
def test_energy_spectrum_matches_oracle(lib, torch_dev, lanes):
    torch, dev = torch_dev
    ns = [100, 256, 300, 777]
    dx, eps = 0.2, 0.02
    p = lib.make_params(dx, 0.05, A, 10)
    plan = lib.Plan(p, ns)
    psis = [ti.random_state(n, 31 + i, width=min(8.0, n * dx / 8), k0=0.5, dx=dx)
            for i, n in enumerate(ns)]
    psi = torch.tensor(np.concatenate([_c2d(x) for x in psis]), device=dev)
    energies = np.linspace(-0.7, 2.5, 41)
    E = torch.tensor(energies, device=dev)
    out = torch.empty(len(ns), len(energies), dtype=torch.float64, device=dev)
    nbytes = lib.tdse_plan_energy_spectrum_work(plan, len(energies), lanes or 65536)
    work = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    print(f"energy spectrum ns={ns} energies={len(energies)} work lanes={lanes}", flush=True)
    lib.tdse_plan_energy_spectrum(plan, psi, E, eps, out, work)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for b, n in enumerate(ns):
        ref = oracle.energy_spectrum(psis[b], energies, eps, dx, A)
        err = np.max(np.abs(got[b] - ref)) / np.max(ref)
        print(f"  n={n}: max err / max P = {err:.3e}", flush=True)
        assert err < 1e-10
    plan.close()


@pytest.mark.parametrize("lanes", [None, 64])
def test_energy_spectrum_blocks_of_many_systems(lib, torch_dev, lanes):
    """Sizes with more systems than a wavefront has lanes (a full block, a
    ragged second block) next to a size with a few: every system against the
    oracle, also with one wavefront of lanes striding over every tile."""
    torch, dev = torch_dev
    ns = [200] * 70 + [333] * 5 + [128] * 64
    dx, eps = 0.2, 0.05
    p = lib.make_params(dx, 0.05, A, 10)
    plan = lib.Plan(p, ns)
    psis = [ti.random_state(n, 500 + i, width=min(6.0, n * dx / 8), k0=0.3, dx=dx)
            for i, n in enumerate(ns)]
    psi = torch.tensor(np.concatenate([_c2d(x) for x in psis]), device=dev)
    energies = np.linspace(-0.6, 1.5, 7)
    E = torch.tensor(energies, device=dev)
    out = torch.empty(len(ns), len(energies), dtype=torch.float64, device=dev)
    nbytes = lib.tdse_plan_energy_spectrum_work(plan, len(energies), lanes or 65536)
    work = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    print(f"energy spectrum blocks: {len(ns)} systems, work lanes={lanes}", flush=True)
    lib.tdse_plan_energy_spectrum(plan, psi, E, eps, out, work)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    worst = 0.0
    for b, n in enumerate(ns):
        ref = oracle.energy_spectrum(psis[b], energies, eps, dx, A)
        worst = max(worst, np.max(np.abs(got[b] - ref)) / np.max(ref))
    print(f"  max err / max P = {worst:.3e}", flush=True)
    assert worst < 1e-10
    plan.close()


def test_energy_integral_and_ionisation_probability(lib, torch_dev):
    """tdse_energy_integral of device spectra against the oracle's trapezoid
    rule on the same values (threshold inside the grid, at -inf and above
    it), and the ionisation probability of propagated states end to end
    against the oracle's (spectrum and integral both on the CPU)."""
    torch, dev = torch_dev
    ns = [300, 512, 300]
    dx, dt, eps = 0.2, 0.05, 0.05
    nt = 400
    p = lib.make_params(dx, dt, A, nt, mask_fraction=0.2)
    plan = lib.Plan(p, ns)
    rng = np.random.default_rng(4)
    efield = 0.06 * np.sin(0.25 * np.arange(nt + 1) * dt)[None, :] * (1.0 + 0.3 * rng.random((3, 1)))
    E = torch.tensor(efield, device=dev)
    acc = torch.empty_like(E)
    pf = torch.empty(2 * sum(ns), dtype=torch.float64, device=dev)
    lib.tdse_propagate_batch(plan, E, None, acc, psi_final=pf)
    energies = np.linspace(-0.7, 2.5, 161)
    Eg = torch.tensor(energies, device=dev)
    spec = torch.empty(len(ns), len(energies), dtype=torch.float64, device=dev)
    nbytes = lib.tdse_plan_energy_spectrum_work(plan, len(energies), 65536)
    work = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    lib.tdse_plan_energy_spectrum(plan, pf, Eg, eps, spec, work)
    out = torch.empty(len(ns), dtype=torch.float64, device=dev)
    sp = None
    for e_lo in (0.0, -np.inf, 0.3, 5.0):
        lib.tdse_energy_integral(Eg, spec, e_lo, out)
        torch.cuda.synchronize()
        sp = spec.cpu().numpy()
        ref = oracle.energy_integral(energies, sp, e_lo)
        got = out.cpu().numpy()
        print(f"energy integral e_lo={e_lo}: {got}", flush=True)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-300)
    lib.tdse_energy_integral(Eg, spec, 0.0, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    psi_f = pf.cpu().numpy().view(np.complex128)
    off = np.concatenate([[0], np.cumsum(ns)])
    for b, n in enumerate(ns):
        ref = oracle.ionisation_probability(psi_f[off[b]:off[b + 1]], energies, eps, dx, A)
        print(f"  n={n}: ionisation probability {got[b]:.6e} (oracle on the GPU state {ref:.6e})", flush=True)
        assert abs(got[b] - ref) <= 1e-10 * abs(ref) + 1e-15
        assert 0.0 < got[b] < 1.0
    plan.close()


def test_eigenstate_lorentzian_and_small_workspace(lib, torch_dev):
    torch, dev = torch_dev
    n, dx, eps = 512, 0.2, 1e-3
    p = lib.make_params(dx, 0.05, A, 10)
    plan = lib.Plan(p, [n])
    psi = torch.empty(2 * n, dtype=torch.float64, device=dev)
    e_g = plan.ground_state(n, psi)
    E = torch.tensor([e_g, e_g + eps, e_g + 3 * eps], dtype=torch.float64, device=dev)
    out = torch.empty(1, 3, dtype=torch.float64, device=dev)
    nbytes = lib.tdse_plan_energy_spectrum_work(plan, 3, 64)
    work = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    lib.tdse_plan_energy_spectrum(plan, psi, E, eps, out, work)
    torch.cuda.synchronize()
    lor = 1.0 / (np.pi * eps) / (1.0 + np.array([0.0, 1.0, 9.0]))
    assert np.max(np.abs(out.cpu().numpy()[0] - lor) / lor) < 1e-6
    with pytest.raises(lib.TDSEError):
        lib.tdse_plan_energy_spectrum(plan, psi, E, eps, out, work[: (nbytes - 16 * n) // 8])
    plan.close()


def test_gabor_matches_oracle(lib, torch_dev):
    """Gabor transform of random rows: centres at the edges and inside,
    more frequencies than threads per workgroup."""
    torch, dev = torch_dev
    rng = np.random.default_rng(21)
    dt, nt, sigma = 0.05, 6000, 8.0
    a = rng.standard_normal((3, nt + 1))
    tc = np.array([0.0, 40.0, 150.0, 299.0, nt * dt])
    om = np.linspace(0.1, 6.0, 300)
    out = torch.empty(3, len(tc), len(om), dtype=torch.float64, device=dev)
    t = lambda x: torch.tensor(np.ascontiguousarray(x), device=dev)
    lib.tdse_gabor(t(a), dt, t(tc), t(om), sigma, out)
    torch.cuda.synchronize()
    ref = oracle.gabor(a, dt, tc, om, sigma)
    err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(ref)
    print(f"gabor: max err / max G = {err:.3e}", flush=True)
    assert err < 1e-10


def test_stored_states_along_a_propagation(lib, torch_dev):
    """The states a storing forward pass keeps every K steps, copied out in
    natural order, equal the oracle's state after the same number of steps;
    from them the time-dependent ground-state population follows."""
    torch, dev = torch_dev
    ns = [256, 400]
    dx, dt, om, nc, K = 0.4, 0.05, 0.25, 2, 37
    nt = ti.n_steps(om, nc, dt)
    efield = ti.sin2_pulse(np.array([0.1, 0.07]), om, nc, dt, nt=nt)
    p = lib.make_params(dx, dt, 1.1, nt, mask_fraction=0.2)
    plan = lib.Plan(p, ns, adjoint_k=K, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    E = torch.tensor(efield, device=dev)
    lib.tdse_propagate_batch(plan, E, None, torch.empty_like(E))
    gen = plan.checkpoint_generation()
    off = plan.psi_offsets()
    psi = torch.empty(2 * sum(ns), dtype=torch.float64, device=dev)
    for index in (0, 2, nt // K):
        lib.tdse_plan_stored_state(plan, gen, index, psi)
        torch.cuda.synchronize()
        got = psi.cpu().numpy().view(np.complex128)
        for b, n in enumerate(ns):
            psi0 = oracle_side.ground_state(n, dx, 1.1)  # the oracle's own
            steps = index * K
            if steps == 0:
                ref = psi0
            else:
                ref = oracle.propagate(efield[b, :steps + 1], psi0, dx, dt, 1.1, mask_frac=0.2,
                                       want_psi=True)["psi_final"]
            r = float(np.linalg.norm(got[off[b]:off[b + 1]] - ref) / np.linalg.norm(ref))
            pop = abs(dx * np.vdot(psi0, got[off[b]:off[b + 1]])) ** 2
            print(f"  step {steps} n={n}: rel {r:.2e}, ground-state population {pop:.6f}", flush=True)
            assert r < 1e-9
    with pytest.raises(lib.TDSEError):
        lib.tdse_plan_stored_state(plan, gen, nt // K + 1, psi)
    lib.tdse_propagate_batch(plan, E, None, torch.empty_like(E))
    with pytest.raises(lib.TDSEError):
        lib.tdse_plan_stored_state(plan, gen, 0, psi)
    plan.close()


def test_time_dependent_ionisation_from_stored_states(lib, torch_dev):
    """The time-dependent ionisation probability along a pulse: the states a
    storing forward pass keeps every K steps, their energy distributions and
    the integral over E >= 0, each on the device, against the oracle's
    ionisation probability of its own state after the same number of steps."""
    torch, dev = torch_dev
    ns = [300, 420]
    dx, dt, om, nc, K, eps = 0.4, 0.05, 0.25, 2, 37, 0.05
    nt = ti.n_steps(om, nc, dt)
    efield = ti.sin2_pulse(np.array([0.12, 0.09]), om, nc, dt, nt=nt)
    p = lib.make_params(dx, dt, 1.1, nt, mask_fraction=0.2)
    plan = lib.Plan(p, ns, adjoint_k=K, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    E = torch.tensor(efield, device=dev)
    lib.tdse_propagate_batch(plan, E, None, torch.empty_like(E))
    gen = plan.checkpoint_generation()
    off = plan.psi_offsets()
    energies = np.linspace(-0.8, 2.0, 113)
    Eg = torch.tensor(energies, device=dev)
    spec = torch.empty(len(ns), len(energies), dtype=torch.float64, device=dev)
    work = torch.empty(lib.tdse_plan_energy_spectrum_work(plan, len(energies), 4096) // 8,
                       dtype=torch.float64, device=dev)
    prob = torch.empty(len(ns), dtype=torch.float64, device=dev)
    psi = torch.empty(2 * sum(ns), dtype=torch.float64, device=dev)
    for index in (0, (nt // K) // 2, nt // K):
        lib.tdse_plan_stored_state(plan, gen, index, psi)
        lib.tdse_plan_energy_spectrum(plan, psi, Eg, eps, spec, work)
        lib.tdse_energy_integral(Eg, spec, 0.0, prob)
        torch.cuda.synchronize()
        got = prob.cpu().numpy()
        for b, n in enumerate(ns):
            psi0 = oracle_side.ground_state(n, dx, 1.1)  # the oracle's own
            steps = index * K
            st = psi0 if steps == 0 else oracle.propagate(
                efield[b, :steps + 1], psi0, dx, dt, 1.1, mask_frac=0.2, want_psi=True)["psi_final"]
            ref = oracle.ionisation_probability(st, energies, eps, dx, 1.1)
            print(f"  step {steps} n={n}: ionisation probability {got[b]:.6e} (oracle {ref:.6e})",
                  flush=True)
            assert abs(got[b] - ref) <= 1e-9 * abs(ref) + 1e-15
    plan.close()


def test_populations_along_a_propagation(lib, torch_dev):
    """Ground-state and volumetric populations of every stored state against
    the oracle's populations of the oracle's state after the same number of
    steps, with the plan's ground state and with a caller's reference; a
    field-free propagation without absorber keeps the ground state's
    populations at 1."""
    torch, dev = torch_dev
    ns = [256, 400, 700]
    dx, dt, om, nc, K, a = 0.4, 0.05, 0.25, 2, 37, 1.1
    nt = ti.n_steps(om, nc, dt)
    nrec = nt // K + 1
    efield = ti.sin2_pulse(np.array([0.1, 0.07, 0.12]), om, nc, dt, nt=nt)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    plan = lib.Plan(p, ns, adjoint_k=K, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    E = torch.tensor(efield, device=dev)
    lib.tdse_propagate_batch(plan, E, None, torch.empty_like(E))
    gen = plan.checkpoint_generation()
    off = plan.psi_offsets()
    radius = 5.1
    gs = torch.full((len(ns), nrec), -1.0, dtype=torch.float64, device=dev)
    vol = torch.full_like(gs, -1.0)
    lib.tdse_plan_populations(plan, gen, radius, gs, vol)
    # a caller's reference: a normalised Gaussian wave packet per system
    ref = np.concatenate([np.exp(-((np.arange(n) - 0.5 * (n - 1)) * dx) ** 2 / 8.0 + 0.3j * np.arange(n))
                          for n in ns])
    for b, n in enumerate(ns):
        r = ref[off[b]:off[b + 1]]
        ref[off[b]:off[b + 1]] = r / np.sqrt(dx * np.sum(np.abs(r) ** 2))
    R = torch.tensor(ref.view(np.float64), device=dev)
    gs_ref = torch.full_like(gs, -1.0)
    lib.tdse_plan_populations(plan, gen, radius, gs_ref, None, psi_ref=R)
    torch.cuda.synchronize()
    g, v, gr = gs.cpu().numpy(), vol.cpu().numpy(), gs_ref.cpu().numpy()
    for b, n in enumerate(ns):
        psi0 = oracle_side.ground_state(n, dx, a)  # the oracle's own
        for s in (0, 1, nrec // 2, nrec - 1):
            steps = s * K
            psi = psi0 if steps == 0 else oracle.propagate(
                efield[b, :steps + 1], psi0, dx, dt, a, mask_frac=0.2, want_psi=True)["psi_final"]
            e_gs, e_vol = oracle.populations(psi, psi0, dx, radius)
            e_gr, _ = oracle.populations(psi, ref[off[b]:off[b + 1]], dx, radius)
            print(f"  n={n} step {steps}: gs {g[b, s]:.12f} ({e_gs:.12f}), vol {v[b, s]:.12f}",
                  flush=True)
            assert abs(g[b, s] - e_gs) <= 1e-9 * max(e_gs, 1e-3)
            assert abs(v[b, s] - e_vol) <= 1e-9 * e_vol
            assert abs(gr[b, s] - e_gr) <= 1e-9 * max(e_gr, 1e-3)
        assert abs(g[b, 0] - 1.0) < 1e-12
    with pytest.raises(lib.TDSEError):
        lib.tdse_plan_populations(plan, gen, radius, None, None)
    with pytest.raises(lib.TDSEError):
        lib.tdse_plan_populations(plan, gen + 1, radius, gs, vol)
    plan.close()
    # field-free, no absorber: the ground state only turns its phase
    p0 = lib.make_params(dx, dt, a, 200, mask_fraction=0.0)
    plan0 = lib.Plan(p0, [512, 300], adjoint_k=20, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    E0 = torch.zeros((2, 201), dtype=torch.float64, device=dev)
    lib.tdse_propagate_batch(plan0, E0, None, torch.empty_like(E0))
    gs0 = torch.empty((2, 11), dtype=torch.float64, device=dev)
    vol0 = torch.empty_like(gs0)
    lib.tdse_plan_populations(plan0, plan0.checkpoint_generation(), 1e6, gs0, vol0)
    torch.cuda.synchronize()
    assert np.max(np.abs(gs0.cpu().numpy() - 1.0)) < 1e-10
    assert np.max(np.abs(vol0.cpu().numpy() - 1.0)) < 1e-10
    plan0.close()
