"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the
same seeded inputs.  Bar: relative L2 <= 1e-9 on the dipole acceleration
(and <norm>, <x>), <= 1e-5 on gradients.  The oracle side computes its own
ground states, soft-core fits and loss gradients (tests/oracle_side.py):
no value from the HIP path is an oracle input."""
import numpy as np
import pytest

import oracle
import oracle_side
import tdse_inputs as ti

pytestmark = pytest.mark.gpu

A_AR = 1.1891671
TOL_ACC = 1e-9
TOL_GRAD = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _to_dev(torch, dev, x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _c2d(psi):
    return np.ascontiguousarray(np.asarray(psi, np.complex128)).view(np.float64)


def _gpu_abar(lib, torch, dev, acc, dt, om, h_lo, h_hi, weights):
    """accel_bar of the weighted harmonic-yield loss, on the GPU."""
    batch, n1 = acc.shape
    k_lo, nk = lib.tdse_harmonic_band(n1 - 1, dt, om, h_lo, h_hi)
    work = torch.empty(2 * batch * max(nk, 1), dtype=torch.float64, device=dev)
    y = torch.empty(batch, dtype=torch.float64, device=dev)
    ab = torch.empty_like(acc)
    lib.tdse_harmonic_yield(batch, n1 - 1, dt, om, h_lo, h_hi, acc,
                            _to_dev(torch, dev, np.asarray(weights, np.float64)), work, y, ab)
    return ab


def test_ground_state_matches_oracle(lib, torch_dev):
    torch, dev = torch_dev
    for n, dx, a in [(2048, 0.2, A_AR), (700, 0.3, 0.9)]:
        print(f"ground state n={n} dx={dx} a={a}", flush=True)
        p = lib.make_params(dx, 0.05, a, 0)
        psi = torch.empty(2 * n, dtype=torch.float64, device=dev)
        e = lib.tdse_ground_state(p, n, 1.0, 20000, 1e-13, psi)
        ref, e_ref, _ = oracle.ground_state(n, dx, a, dtau=1.0, tol=1e-13)
        got = psi.cpu().numpy().view(np.complex128)
        assert abs(e - e_ref) < 1e-12
        assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_soft_core_fit_reaches_ip(lib, torch_dev):
    print("soft-core fit n=2048", flush=True)
    a, e = lib.tdse_soft_core_for_ip(ti.IP_ARGON, 2048, 0.2, dtau=1.0, tol=1e-13)
    assert abs(e + ti.IP_ARGON) < 1e-13
    # the oracle's own bisection lands on the same parameter
    a_ref = oracle_side.soft_core(ti.IP_ARGON, 0.2)
    print(f"  a = {a:.15f}, oracle {a_ref:.15f}", flush=True)
    assert abs(a - a_ref) < 1e-10


def _run_forward(lib, torch, dev, ns, efield, dx, dt, a, psi0_list=None, mask=0.1, options=0,
                 want=True):
    nt = efield.shape[1] - 1
    p = lib.make_params(dx, dt, a, nt, mask_fraction=mask)
    plan = lib.Plan(p, ns, options=options)
    E = _to_dev(torch, dev, efield)
    acc = torch.empty_like(E)
    xe = torch.empty_like(E) if want else None
    nr = torch.empty_like(E) if want else None
    st = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
    psi0 = None
    if psi0_list is not None:
        psi0 = _to_dev(torch, dev, np.concatenate([_c2d(x) for x in psi0_list]))
    pf = torch.empty(2 * sum(ns), dtype=torch.float64, device=dev)
    lib.tdse_propagate_batch(plan, E, psi0, acc, xe, nr, pf, st)
    torch.cuda.synchronize()
    out = dict(accel=acc.cpu().numpy(), status=st.cpu().numpy(), psi_final=pf.cpu().numpy())
    if want:
        out.update(xexp=xe.cpu().numpy(), norm=nr.cpu().numpy())
    return plan, out


def test_forward_ragged_small_batch_vs_oracle(lib, torch_dev):
    """Several sizes in one batch (several tiles, ragged tails), explicit psi0."""
    torch, dev = torch_dev
    ns = [100, 256, 300, 777, 1024, 2048, 2500, 4096]
    dx, dt = 0.2, 0.05
    om, nc = 0.057, 1
    nt = ti.n_steps(om, nc, dt)
    e0 = np.linspace(0.03, 0.09, len(ns))
    efield = ti.sin2_pulse(e0, om, nc, dt, nt=nt)
    psi0 = [ti.random_state(n, 11 + i, width=min(10.0, n * dx / 8), k0=0.3, dx=dx)
            for i, n in enumerate(ns)]
    print(f"forward ragged ns={ns} nt={nt}", flush=True)
    plan, out = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR, psi0)
    off = plan.psi_offsets()
    pf = out["psi_final"].view(np.complex128)
    for b, n in enumerate(ns):
        ref = oracle.propagate(efield[b], psi0[b], dx, dt, A_AR, mask_frac=0.1, want_psi=True)
        assert out["status"][b] == 0
        assert rel(out["accel"][b], ref["accel"]) < TOL_ACC, (n, rel(out["accel"][b], ref["accel"]))
        assert rel(out["xexp"][b], ref["xexp"]) < TOL_ACC
        assert rel(out["norm"][b], ref["norm"]) < TOL_ACC
        assert rel(pf[off[b]:off[b + 1]], ref["psi_final"]) < TOL_ACC


def test_forward_single_2048_full_pulse(lib, torch_dev):
    """Single-system workload: N = 2048, dx = 0.2, dt = 0.05, 10-cycle 800 nm
    pulse at 1.5e14 W/cm^2 (22 047 steps), plan ground state."""
    torch, dev = torch_dev
    w = ti.cfg1_single()
    efield = w.efield()
    print(f"forward single-2048 nt={w.nt}", flush=True)
    plan, out = _run_forward(lib, torch, dev, [2048], efield, w.dx, w.dt, A_AR)
    ref = oracle_side.propagate(efield[0], 2048, w.dx, w.dt, A_AR, mask_frac=0.1)
    r = rel(out["accel"][0], ref["accel"])
    print(f"  accel rel-L2 {r:.3e}", flush=True)
    assert r < TOL_ACC
    assert rel(out["norm"][0], ref["norm"]) < TOL_ACC


def test_phase_increment_branches_match_oracle(lib, torch_dev):
    """The per-point phase increment dt E dx takes a short series for
    |dt E dx| <= 1e-3, a longer one up to 0.05 and the reduced-range sincos
    beyond: fields ramping through all three ranges (dt = 0.05, dx = 0.2:
    E up to 0.05, 1.0 and 8.0) against the oracle, which evaluates
    exp(-i dt E x_j) point by point."""
    torch, dev = torch_dev
    ns = [1024, 2048, 1500]
    dx, dt, nt = 0.2, 0.05, 300
    ramp = np.linspace(0.0, 1.0, nt + 1)
    efield = np.stack([0.05 * ramp, 1.0 * ramp, 8.0 * ramp])
    print(f"phase increment branches ns={ns} nt={nt} |dt E dx| up to "
          f"{[float(dt * e * dx) for e in (0.05, 1.0, 8.0)]}", flush=True)
    _, out = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR)
    assert np.all(out["status"] == 0)
    for b, n in enumerate(ns):
        ref = oracle_side.propagate(efield[b], n, dx, dt, A_AR, mask_frac=0.1)
        r = rel(out["accel"][b], ref["accel"])
        print(f"  system {b}: accel rel-L2 {r:.3e}", flush=True)
        assert r < TOL_ACC
        assert rel(out["norm"][b], ref["norm"]) < TOL_ACC


def test_plan_ground_state_matches_oracle(lib, torch_dev):
    torch, dev = torch_dev
    p = lib.make_params(0.2, 0.05, A_AR, 10)
    plan = lib.Plan(p, [2048, 1000])
    for n in (2048, 1000):
        psi = torch.empty(2 * n, dtype=torch.float64, device=dev)
        e = plan.ground_state(n, psi)
        ref, e_ref, _ = oracle.ground_state(n, 0.2, A_AR, dtau=1.0, tol=1e-13)
        assert abs(e - e_ref) < 1e-12
        assert np.max(np.abs(psi.cpu().numpy().view(np.complex128) - ref)) < 1e-9


def test_plain_graph_direct_identical(lib, torch_dev):
    """Plain (one launch per system), direct launches and graph replays give
    bitwise identical outputs; repeated graph replays too."""
    torch, dev = torch_dev
    ns = [512, 512, 1024, 300]
    nt = 300
    rng = np.random.default_rng(3)
    efield = 0.05 * rng.standard_normal((len(ns), nt + 1))
    outs = []
    for opt in (lib.TDSE_OPT_PLAIN, lib.TDSE_OPT_NO_GRAPH, 0):
        print(f"options={opt}", flush=True)
        outs.append(_run_forward(lib, torch, dev, ns, efield, 0.2, 0.05, A_AR, options=opt)[1])
    for o in outs[1:]:
        assert np.array_equal(o["accel"], outs[0]["accel"])
        assert np.array_equal(o["psi_final"], outs[0]["psi_final"])
    p = lib.make_params(0.2, 0.05, A_AR, nt)
    plan = lib.Plan(p, ns)
    E = _to_dev(torch, dev, efield)
    accs = []
    for rep in range(3):
        acc = torch.empty_like(E) if rep == 0 else accs[0][1]
        lib.tdse_propagate_batch(plan, E, None, acc)
        torch.cuda.synchronize()
        accs.append((acc.cpu().numpy().copy(), acc))
        torch.cuda.synchronize()
    for a_, _ in accs[1:]:
        assert np.array_equal(a_, accs[0][0])
    assert np.array_equal(accs[0][0], outs[0]["accel"])


def test_nonfinite_field_is_flagged(lib, torch_dev):
    torch, dev = torch_dev
    nt = 100
    efield = np.zeros((2, nt + 1))
    efield[1, 40] = np.nan
    _, out = _run_forward(lib, torch, dev, [256, 256], efield, 0.2, 0.05, A_AR)
    assert out["status"][0] == 0
    assert out["status"][1] & lib.TDSE_SYS_NONFINITE


def test_invalid_arguments_are_refused_before_any_launch(lib, torch_dev):
    """Argument errors come back as TDSE_E_INVALID / TDSE_E_UNSUPPORTED with a
    detail message, and leave the plan usable."""
    torch, dev = torch_dev
    nt = 40
    p = lib.make_params(0.4, 0.05, 1.1, nt, mask_fraction=0.2)

    def status_of(fn):
        with pytest.raises(lib.TDSEError) as ei:
            fn()
        assert str(ei.value)
        return ei.value.status

    assert status_of(lambda: lib.Plan(p, [])) == lib.TDSE_E_INVALID               # empty batch
    assert status_of(lambda: lib.Plan(p, [8])) == lib.TDSE_E_INVALID              # n < 16
    assert status_of(lambda: lib.Plan(p, [20000])) == lib.TDSE_E_UNSUPPORTED      # n > 16384
    assert status_of(lambda: lib.Plan(p, [256], options=64)) == lib.TDSE_E_INVALID
    assert status_of(lambda: lib.Plan(p, [256], options=lib.TDSE_OPT_STORE_CHECKPOINTS)) \
        == lib.TDSE_E_INVALID                                                    # needs adjoint_k
    bad = lib.make_params(-0.4, 0.05, 1.1, nt)
    assert status_of(lambda: lib.Plan(bad, [256])) == lib.TDSE_E_INVALID
    plan = lib.Plan(p, [256, 300])
    E = torch.zeros(2, nt + 1, dtype=torch.float64, device=dev)
    acc = torch.empty_like(E)
    assert status_of(lambda: lib.tdse_propagate_batch(plan, E, None, None)) == lib.TDSE_E_INVALID
    flat = torch.zeros(2 * (nt + 1) + 1, dtype=torch.float64, device=dev)
    assert status_of(lambda: lib.tdse_propagate_batch(plan, E, None, flat[1:])) \
        == lib.TDSE_E_INVALID                                                    # misaligned
    assert status_of(lambda: lib.tdse_adjoint_batch(plan, E, None, acc, acc)) == lib.TDSE_E_INVALID
    assert status_of(lambda: lib.tdse_adjoint_batch_stored(plan, 1, E, acc, acc)) \
        == lib.TDSE_E_INVALID
    lib.tdse_propagate_batch(plan, E, None, acc)      # still usable
    torch.cuda.synchronize()
    assert torch.isfinite(acc).all()
    plan.close()


@pytest.mark.parametrize("nt", [0, 1, 5, 32, 33])
def test_degenerate_lengths_and_layout_boundaries(lib, torch_dev, nt):
    """Propagations of 0, 1, 5, 32 and 33 steps (checkpoint interval longer
    than the run, and one checkpoint per step; 32 and 33 end exactly on and
    one step past a block of the forward kernel's 32-step output flush and
    phase-ratio fill) on the smallest grid and on both sides of every layout
    boundary (4 | 8 points per lane at 512, 8 | 16 at 8192): outputs, final
    states and gradients, recomputed and from stored checkpoints, against the
    oracle."""
    torch, dev = torch_dev
    ns = [16, 17, 511, 512, 513, 8192, 8193]
    dx, dt, a = 0.4, 0.05, 1.1
    rng = np.random.default_rng(100 + nt)
    efield = 0.05 * rng.standard_normal((len(ns), nt + 1))
    abar = rng.standard_normal((len(ns), nt + 1))
    E, AB = _to_dev(torch, dev, efield), _to_dev(torch, dev, abar)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    for k in (256, 1):
        print(f"degenerate ns={ns} nt={nt} K={k}", flush=True)
        plan = lib.Plan(p, ns, adjoint_k=k, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
        acc, xe, nr = (torch.empty_like(E) for _ in range(3))
        pf = torch.empty(2 * sum(ns), dtype=torch.float64, device=dev)
        st = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
        lib.tdse_propagate_batch(plan, E, None, acc, xe, nr, pf, st)
        g_st = torch.full_like(E, 7.0)
        lib.tdse_adjoint_batch_stored(plan, plan.checkpoint_generation(), E, AB, g_st)
        g = torch.full_like(E, 7.0)
        lib.tdse_adjoint_batch(plan, E, None, AB, g)
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == 0)
        assert np.array_equal(g.cpu().numpy(), g_st.cpu().numpy())
        off = plan.psi_offsets()
        got = {key: t.cpu().numpy() for key, t in (("accel", acc), ("xexp", xe), ("norm", nr))}
        pfin = pf.cpu().numpy().view(np.complex128)
        gg = g.cpu().numpy()
        for b, n in enumerate(ns):
            ref = oracle_side.propagate(efield[b], n, dx, dt, a, mask_frac=0.2, want_psi=True)
            g_ref, _ = oracle_side.adjoint(efield[b], abar[b], n, dx, dt, a, mask_frac=0.2, k=k)
            for key in ("accel", "norm"):
                assert rel(got[key][b], ref[key]) < TOL_ACC, (n, key)
            # <x> is zero by symmetry at t = 0: compare on the scale of the grid
            assert np.max(np.abs(got["xexp"][b] - ref["xexp"])) < TOL_ACC * n * dx
            assert rel(pfin[off[b]:off[b + 1]], ref["psi_final"]) < TOL_ACC
            assert rel(gg[b], g_ref) < 1e-9, (n, k)
        plan.close()


def test_harmonic_yield_matches_oracle(lib, torch_dev):
    torch, dev = torch_dev
    rng = np.random.default_rng(4)
    nt, dt, om = 4000, 0.05, 0.057
    t = np.arange(nt + 1) * dt
    acc = np.sin(0.057 * 25 * t)[None, :] * rng.uniform(0.5, 1.5, (3, 1)) + 1e-3 * rng.standard_normal((3, nt + 1))
    w = np.array([1.0, 0.0, 2.0])
    k_lo, nk = lib.tdse_harmonic_band(nt, dt, om, 21, 31)
    A = _to_dev(torch, dev, acc)
    Wt = _to_dev(torch, dev, w)
    work = torch.empty(2 * 3 * max(nk, 1), dtype=torch.float64, device=dev)
    y = torch.empty(3, dtype=torch.float64, device=dev)
    ab = torch.empty_like(A)
    lib.tdse_harmonic_yield(3, nt, dt, om, 21, 31, A, Wt, work, y, ab)
    torch.cuda.synchronize()
    l_ref, ab_ref = oracle.harmonic_yield(acc, dt, om, 21, 31)
    assert np.allclose(y.cpu().numpy(), w * l_ref, rtol=1e-11, atol=0)
    got = ab.cpu().numpy()
    for b in (0, 2):
        assert rel(got[b], w[b] * ab_ref[b]) < 1e-10
    assert np.all(got[1] == 0.0)


def test_adjoint_matches_oracle_and_fd(lib, torch_dev):
    torch, dev = torch_dev
    ns = [256, 256, 400]
    dx, dt, a = 0.4, 0.05, 1.1
    om, nc = 0.25, 3
    nt = ti.n_steps(om, nc, dt)
    e0 = np.array([0.1, 0.12, 0.0])
    efield = ti.sin2_pulse(e0, om, nc, dt, nt=nt)
    efield[2] = 0.05 * np.random.default_rng(7).standard_normal(nt + 1)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    for k in (37, 256):
        print(f"adjoint ns={ns} nt={nt} K={k}", flush=True)
        plan = lib.Plan(p, ns, adjoint_k=k)
        E = _to_dev(torch, dev, efield)
        acc = torch.empty_like(E)
        lib.tdse_propagate_batch(plan, E, None, acc)
        # an all-zero row (weight 0) is skipped
        AB = _gpu_abar(lib, torch, dev, acc, dt, om, 3, 9, [1.0, 0.0, 1.0])
        grad = torch.full_like(E, 7.0)
        acc2 = torch.empty_like(E)
        st = torch.full((3,), -1, dtype=torch.int32, device=dev)
        lib.tdse_adjoint_batch(plan, E, None, AB, grad, acc2, st)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        assert np.array_equal(acc2.cpu().numpy(), acc.cpu().numpy())
        assert np.all(st.cpu().numpy() == 0)
        assert np.all(g[1] == 0.0)
        for b in (0, 2):
            _, g_ref = oracle_side.yield_gradient(efield[b], ns[b], dx, dt, a, om, 3, 9,
                                                  mask_frac=0.2, k=k)
            r = rel(g[b], g_ref)
            print(f"  grad rel-L2 system {b}: {r:.3e}", flush=True)
            assert r < 1e-9
        plan.close()


def test_adjoint_across_layouts(lib, torch_dev):
    """The adjoint at 8 and 16 points per lane (N = 700, 9000 and the maximum
    16384, where the 16-point kernel parks the costate while a segment is
    recomputed and streams psi from the segment buffer), recomputing and from
    stored checkpoints: bitwise equal to each other and within the bar of the
    oracle's adjoint."""
    torch, dev = torch_dev
    ns = [700, 9000, 16384]
    dx, dt, a, nt, k = 0.4, 0.05, 1.1, 240, 37
    rng = np.random.default_rng(11)
    efield = 0.05 * rng.standard_normal((len(ns), nt + 1))
    abar = rng.standard_normal((len(ns), nt + 1))
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    E, AB = _to_dev(torch, dev, efield), _to_dev(torch, dev, abar)
    print(f"adjoint layouts ns={ns} nt={nt} K={k}", flush=True)
    ref = lib.Plan(p, ns, adjoint_k=k)
    stp = lib.Plan(p, ns, adjoint_k=k, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    assert [ref.layout(n).points_per_lane for n in ns] == [8, 16, 16]
    g_full = torch.full_like(E, 7.0)
    acc = torch.empty_like(E)
    st = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
    lib.tdse_adjoint_batch(ref, E, None, AB, g_full, acc, st)
    lib.tdse_propagate_batch(stp, E, None, torch.empty_like(E))
    g_st = torch.full_like(E, 7.0)
    lib.tdse_adjoint_batch_stored(stp, stp.checkpoint_generation(), E, AB, g_st)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    g, acc_np = g_full.cpu().numpy(), acc.cpu().numpy()
    assert np.array_equal(g_st.cpu().numpy(), g)
    for b, n in enumerate(ns):
        g_ref, acc_ref = oracle_side.adjoint(efield[b], abar[b], n, dx, dt, a, mask_frac=0.2, k=k)
        r, ra = rel(g[b], g_ref), rel(acc_np[b], acc_ref)
        print(f"  n={n}: grad rel-L2 {r:.3e}, accel rel-L2 {ra:.3e}", flush=True)
        assert r < 1e-9 and ra < TOL_ACC
    ref.close()
    stp.close()


def test_stored_checkpoints_match_recomputing_adjoint(lib, torch_dev):
    """A plan that stores the adjoint checkpoints in its forward pass gives
    the same forward outputs as a plain plan of the same layouts, its reverse
    sweep from the stored checkpoints gives the recomputing adjoint's
    gradient bitwise (and the oracle's), and a stale generation is refused."""
    torch, dev = torch_dev
    ns = [256, 400, 256]
    dx, dt, a = 0.4, 0.05, 1.1
    om, nc = 0.25, 3
    nt = ti.n_steps(om, nc, dt)
    efield = ti.sin2_pulse(np.array([0.1, 0.12, 0.08]), om, nc, dt, nt=nt)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    E = _to_dev(torch, dev, efield)
    print(f"stored checkpoints ns={ns} nt={nt} K=37", flush=True)
    ref = lib.Plan(p, ns, adjoint_k=37)
    stp = lib.Plan(p, ns, adjoint_k=37, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    assert stp.checkpoint_generation() == 0
    outs = []
    for pl in (ref, stp):
        acc, xe, nr = (torch.empty_like(E) for _ in range(3))
        pf = torch.empty(2 * sum(ns), dtype=torch.float64, device=dev)
        status = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
        lib.tdse_propagate_batch(pl, E, None, acc, xe, nr, pf, status)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (acc, xe, nr, pf, status)])
    gen = stp.checkpoint_generation()
    assert gen == 1
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)
    assert np.all(outs[1][4] == 0)
    # an all-zero row (weight 0) is skipped here too
    AB = _gpu_abar(lib, torch, dev, _to_dev(torch, dev, outs[0][0]), dt, om, 3, 9, [1.0, 0.0, 1.0])
    g_full = torch.full_like(E, 7.0)
    lib.tdse_adjoint_batch(ref, E, None, AB, g_full)
    g_st = torch.full_like(E, 7.0)
    st = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
    lib.tdse_adjoint_batch_stored(stp, gen, E, AB, g_st, st)
    torch.cuda.synchronize()
    assert np.array_equal(g_st.cpu().numpy(), g_full.cpu().numpy())
    assert np.all(st.cpu().numpy() == 0)
    assert np.all(g_st.cpu().numpy()[1] == 0.0)
    _, g_ref = oracle_side.yield_gradient(efield[2], ns[2], dx, dt, a, om, 3, 9, mask_frac=0.2,
                                          k=37)
    assert rel(g_st.cpu().numpy()[2], g_ref) < 1e-9
    # a later forward pass rewrites the store: the old generation is refused
    lib.tdse_propagate_batch(stp, E, None, torch.empty_like(E))
    with pytest.raises(lib.TDSEError):
        lib.tdse_adjoint_batch_stored(stp, gen, E, AB, g_st)
    # the recomputing adjoint works on the storing plan and rewrites the store
    g2 = torch.full_like(E, 7.0)
    lib.tdse_adjoint_batch(stp, E, None, AB, g2)
    torch.cuda.synchronize()
    assert np.array_equal(g2.cpu().numpy(), g_full.cpu().numpy())
    assert stp.checkpoint_generation() == gen + 2
    ref.close()
    stp.close()


def test_table_placement_does_not_change_results(lib, torch_dev, monkeypatch):
    """The per-point tables staged in LDS (both, or om alone) or read from
    global memory hold the same values, so every placement gives bitwise
    the same outputs (TDSE_PACK_LDS forces a placement at plan creation)."""
    torch, dev = torch_dev
    dx, dt = 0.2, 0.05
    nt = 60
    for ns, forced in (([600, 2048, 3000], "0"), ([9000, 12000], "0"), ([9000, 12000], "2")):
        efield = ti.sin2_pulse(np.linspace(0.05, 0.08, len(ns)), 0.057, 1, dt, nt=nt)
        monkeypatch.delenv("TDSE_PACK_LDS", raising=False)
        plan_d, ref = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR)
        placement_d = [plan_d.launch_info(n).lds_tables for n in ns]
        monkeypatch.setenv("TDSE_PACK_LDS", forced)
        plan_f, out = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR)
        placement_f = [plan_f.launch_info(n).lds_tables for n in ns]
        monkeypatch.delenv("TDSE_PACK_LDS")
        print(f"placement ns={ns}: default {placement_d}, forced {placement_f}", flush=True)
        assert placement_f == [int(forced)] * len(ns)
        for key in ("accel", "xexp", "norm", "psi_final"):
            assert np.array_equal(out[key], ref[key]), key
        plan_d.close()
        plan_f.close()


def test_narrow_instances_match_wide_bitwise(lib, torch_dev, monkeypatch):
    """Workgroups of at most 512 threads run the narrow forward instances
    (256 registers per lane; at 16 points per lane with q in registers and
    the elimination factors formed from it).  Packed into 1024-thread
    workgroups instead, the same systems run the wide instances: plain and
    population outputs bitwise equal, and within the bar of the oracle."""
    torch, dev = torch_dev
    dx, dt, nt = 0.2, 0.05, 300
    for C, count, narrow_s in ((8, 6, "2"), (16, 8, "4")):
        ns = [2000] * count
        efield = ti.sin2_pulse(np.linspace(0.05, 0.08, count), 0.057, 1, dt, nt=nt)
        monkeypatch.setenv("TDSE_LAYOUT_C", str(C))
        monkeypatch.delenv("TDSE_PACK_S", raising=False)
        plan_w, out_w = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR)
        monkeypatch.setenv("TDSE_PACK_S", narrow_s)
        plan_n, out_n = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR)
        monkeypatch.delenv("TDSE_PACK_S")
        monkeypatch.delenv("TDSE_LAYOUT_C")
        kw, kn = plan_w.kernel_info(2000), plan_n.kernel_info(2000)
        print(f"C={C}: wide {kw.workgroup_lanes} lanes {kw.vgprs} VGPRs, "
              f"narrow {kn.workgroup_lanes} lanes {kn.vgprs} VGPRs", flush=True)
        assert plan_n.layout(2000).points_per_lane == C
        assert kw.workgroup_lanes == 1024 and kn.workgroup_lanes == 512
        assert kn.vgprs > 128
        for key in ("accel", "xexp", "norm", "psi_final"):
            assert np.array_equal(out_n[key], out_w[key]), key
        assert np.all(out_n["status"] == 0)
        # the population variant of the same kernels
        pops = []
        for plan in (plan_w, plan_n):
            E = _to_dev(torch, dev, efield)
            acc, gs, vol = (torch.empty_like(E) for _ in range(3))
            lib.tdse_propagate_batch_populations(plan, E, None, acc, 5.0, gs, vol)
            torch.cuda.synchronize()
            pops.append([t.cpu().numpy() for t in (acc, gs, vol)])
        for x, y in zip(*pops):
            assert np.array_equal(x, y)
        ref = oracle_side.propagate(efield[0], 2000, dx, dt, A_AR, mask_frac=0.1)
        assert rel(out_n["accel"][0], ref["accel"]) < TOL_ACC
        plan_w.close()
        plan_n.close()


def test_elimination_factor_source_does_not_change_results(lib, torch_dev, monkeypatch):
    """Layouts without q in registers (16 points per lane forward, 8 and 16
    in the adjoint) read alpha and beta from their tables, or form them from
    q and om (TDSE_AB_TABLES=0): the tables hold the kernels' own values, so
    both give bitwise the same forward outputs and gradients, and the
    oracle's."""
    torch, dev = torch_dev
    ns = [3000, 9000, 12000]
    dx, dt, a, nt, k = 0.2, 0.05, A_AR, 150, 40
    rng = np.random.default_rng(31)
    efield = 0.06 * rng.standard_normal((len(ns), nt + 1))
    abar = rng.standard_normal((len(ns), nt + 1))
    E, AB = _to_dev(torch, dev, efield), _to_dev(torch, dev, abar)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.1)
    res = {}
    for budget in (None, "0"):
        if budget is None:
            monkeypatch.delenv("TDSE_AB_TABLES", raising=False)
        else:
            monkeypatch.setenv("TDSE_AB_TABLES", budget)
        plan = lib.Plan(p, ns, adjoint_k=k)
        monkeypatch.delenv("TDSE_AB_TABLES", raising=False)
        acc = torch.empty_like(E)
        g = torch.empty_like(E)
        lib.tdse_propagate_batch(plan, E, None, acc)
        lib.tdse_adjoint_batch(plan, E, None, AB, g)
        torch.cuda.synchronize()
        res[budget] = (acc.cpu().numpy(), g.cpu().numpy())
        print(f"  TDSE_AB_TABLES={budget}: layouts {[plan.layout(n).points_per_lane for n in ns]}", flush=True)
        plan.close()
    for b, n in enumerate(ns):
        r_acc = rel(res[None][0][b], res["0"][0][b])
        r_g = rel(res[None][1][b], res["0"][1][b])
        print(f"  n={n}: tables vs formed: accel {r_acc:.2e}, grad {r_g:.2e}", flush=True)
        assert r_acc == 0.0 and r_g == 0.0
    for b in (1, 2):
        g_ref, acc_ref = oracle_side.adjoint(efield[b], abar[b], ns[b], dx, dt, a, mask_frac=0.1,
                                             k=k)
        for key in (None, "0"):
            assert rel(res[key][0][b], acc_ref) < TOL_ACC
            assert rel(res[key][1][b], g_ref) < 1e-9


def test_twelve_points_per_lane(lib, torch_dev, monkeypatch):
    """The 12-point layout (forward only; chosen by the autotuner where it
    fills workgroups better than 16 points, e.g. N = 12288 = 12 x 1024),
    forced here for every size: outputs against the oracle, statuses clean."""
    torch, dev = torch_dev
    ns = [3000, 9000, 12288]
    dx, dt, nt = 0.2, 0.05, 300
    efield = 0.06 * np.random.default_rng(41).standard_normal((len(ns), nt + 1))
    monkeypatch.setenv("TDSE_LAYOUT_C", "12")
    plan, out = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR)
    monkeypatch.delenv("TDSE_LAYOUT_C")
    assert [plan.layout(n).points_per_lane for n in ns] == [12, 12, 12]
    assert np.all(out["status"] == 0)
    off = plan.psi_offsets()
    pf = out["psi_final"].view(np.complex128)
    for b, n in enumerate(ns):
        ref = oracle_side.propagate(efield[b], n, dx, dt, A_AR, mask_frac=0.1, want_psi=True)
        r = rel(out["accel"][b], ref["accel"])
        print(f"  n={n} lanes={plan.layout(n).lanes}: accel rel-L2 {r:.3e}", flush=True)
        assert r < TOL_ACC
        assert rel(out["norm"][b], ref["norm"]) < TOL_ACC
        assert rel(pf[off[b]:off[b + 1]], ref["psi_final"]) < TOL_ACC
    plan.close()


def test_forward_uneven_wide_batch_sampled(lib, torch_dev):
    """Uneven batch spanning N = 2048..16384 (many size classes; tables in
    LDS, om alone in LDS; 8 and 16 points per lane), first 400 steps of the
    1300 nm pulse; sampled systems against the oracle, all statuses clean."""
    torch, dev = torch_dev
    w = ti.cfg3_uneven(batch=96, wide=True)
    nt = 400
    efield = np.ascontiguousarray(w.efield()[:, :nt + 1])
    ns = w.n_per
    order = np.argsort(ns)
    picks = sorted({int(order[0]), int(order[len(ns) // 3]), int(order[len(ns) // 2]),
                    int(order[-2]), int(order[-1])})
    print(f"uneven-wide batch={len(ns)} classes={len(set(ns))} n=[{min(ns)},{max(ns)}] nt={nt}",
          flush=True)
    plan, out = _run_forward(lib, torch, dev, ns, efield, w.dx, w.dt, A_AR, want=False)
    assert np.all(out["status"] == 0)
    for b in picks:
        ref = oracle_side.propagate(efield[b], ns[b], w.dx, w.dt, A_AR, mask_frac=0.1)
        r = rel(out["accel"][b], ref["accel"])
        print(f"  system {b} n={ns[b]} layout={plan.layout(ns[b])}: accel rel-L2 {r:.3e}", flush=True)
        assert r < TOL_ACC
    plan.close()


def test_uneven_wide_autotuned_groups_graph_equals_direct(lib, torch_dev):
    """The whole wide uneven batch (4096 systems, 57 sizes), autotuned as the
    benchmark runs it: more lane-layout groups than graph branches, so one
    branch carries two launches in the plan's launch order.  The graph
    replay equals direct launches on one stream bitwise, every status is
    clean, and sampled systems of the smallest, a 12-point and the largest
    grid match the oracle over the first 1000 steps.  (The acceleration
    grows as t^2 at the start of the sin^2 envelope, while the two sides'
    independently relaxed ground states leave a fixed absolute difference:
    over the first 160 steps that floor alone is 1.5e-9 of the signal, over
    400 steps 2.6e-10, over 1000 steps 7e-11.)"""
    torch, dev = torch_dev
    w = ti.cfg3_uneven(wide=True)
    nt = 1000
    efield = np.ascontiguousarray(w.efield(nt=nt))
    ns = [int(n) for n in w.n_per]
    outs = []
    for opt in (lib.TDSE_OPT_AUTOTUNE, lib.TDSE_OPT_AUTOTUNE | lib.TDSE_OPT_NO_GRAPH):
        print(f"uneven-wide batch={len(ns)} classes={len(set(ns))} nt={nt} options={opt}", flush=True)
        plan, out = _run_forward(lib, torch, dev, ns, efield, w.dx, w.dt, A_AR, options=opt,
                                 want=False)
        groups = {(plan.layout(n).points_per_lane, plan.launch_info(n).lds_tables) for n in set(ns)}
        lay = {n: plan.layout(n).points_per_lane for n in set(ns)}
        outs.append(out)
        plan.close()
        print(f"  layout groups (points per lane, tables): {sorted(groups)}", flush=True)
        assert len(groups) > 4
        assert np.all(out["status"] == 0)
    assert np.array_equal(outs[0]["accel"], outs[1]["accel"])
    assert np.array_equal(outs[0]["psi_final"], outs[1]["psi_final"])
    twelve = [b for b, n in enumerate(ns) if lay[n] == 12]
    picks = [int(np.argmin(ns)), twelve[0], int(np.argmax(ns))]
    for b in picks:
        ref = oracle_side.propagate(efield[b], ns[b], w.dx, w.dt, A_AR, mask_frac=0.1)
        r = rel(outs[0]["accel"][b], ref["accel"])
        print(f"  system {b} n={ns[b]} C={lay[ns[b]]}: accel rel-L2 {r:.3e}", flush=True)
        assert r < TOL_ACC


def test_focus_batch_full_size_sampled(lib, torch_dev):
    """The benchmark workload at its full size and in the benchmark's launch
    configuration (1024 systems x 4096 points x 44093 steps, autotuned plan,
    graph replay): two sampled systems (the hottest and one off-axis) against
    the oracle over the whole pulse, every status clean, norms non-increasing."""
    torch, dev = torch_dev
    w = ti.cfg2_focus()
    a_sc, _ = lib.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    p = lib.make_params(w.dx, w.dt, a_sc, w.nt, mask_fraction=w.mask_frac, mask_power=w.mask_pow)
    plan = lib.Plan(p, w.n_per, options=lib.TDSE_OPT_AUTOTUNE)
    E = w.efield(xp={"device": dev}).contiguous()
    acc = torch.empty_like(E)
    nr = torch.empty_like(E)
    st = torch.full((w.batch,), -1, dtype=torch.int32, device=dev)
    print(f"focus full size: {w.batch} x {w.n_per[0]} x {w.nt}", flush=True)
    lib.tdse_propagate_batch(plan, E, None, acc, None, nr, None, st)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    assert bool((nr[:, 1:] <= nr[:, :-1] * (1 + 1e-12)).all())
    # the oracle's own soft-core fit and ground state
    a_ref = oracle_side.soft_core(w.ip, w.dx)
    psi0 = oracle_side.ground_state(w.n_per[0], w.dx, a_ref)
    rows = [int(np.argmax(w.e0)), w.batch - 1]
    ref = oracle.propagate_batch(w.efield(rows=rows), [psi0, psi0], w.dx, w.dt, a_ref,
                                 mask_frac=w.mask_frac, mask_pow=w.mask_pow, nthreads=2)
    got = acc[rows].cpu().numpy()
    for i, r in enumerate(rows):
        e = rel(got[i], ref["accel"][i])
        print(f"  system {r}: accel rel-L2 {e:.3e}", flush=True)
        assert e < TOL_ACC
    plan.close()


def test_uneven_workload_full_size_sampled(lib, torch_dev):
    """The uneven workload at its full size in the benchmark's launch
    configuration (4096 systems, six grid sizes 2048-3328 sharing
    workgroups, 85 924 steps, autotuned plan, graph replay): the systems with
    the smallest and the largest grid against the oracle over the whole
    pulse, every status clean."""
    from concurrent.futures import ThreadPoolExecutor

    torch, dev = torch_dev
    w = ti.cfg3_uneven()
    a_sc, _ = lib.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    p = lib.make_params(w.dx, w.dt, a_sc, w.nt, mask_fraction=w.mask_frac, mask_power=w.mask_pow)
    plan = lib.Plan(p, w.n_per, options=lib.TDSE_OPT_AUTOTUNE)
    E = w.efield(xp={"device": dev}).contiguous()
    acc = torch.empty_like(E)
    st = torch.full((w.batch,), -1, dtype=torch.int32, device=dev)
    print(f"uneven full size: {w.batch} systems, n {min(w.n_per)}-{max(w.n_per)}, nt={w.nt}",
          flush=True)
    lib.tdse_propagate_batch(plan, E, None, acc, None, None, None, st)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    order = np.argsort(w.n_per, kind="stable")
    rows = [int(order[0]), int(order[-1])]
    a_ref = oracle_side.soft_core(w.ip, w.dx)
    e_rows = w.efield(rows=rows)
    with ThreadPoolExecutor(len(rows)) as ex:
        refs = list(ex.map(lambda i: oracle_side.propagate(
            e_rows[i], w.n_per[rows[i]], w.dx, w.dt, a_ref, mask_frac=w.mask_frac,
            mask_pow=w.mask_pow)["accel"], range(len(rows))))
    got = acc[rows].cpu().numpy()
    for i, r in enumerate(rows):
        e = rel(got[i], refs[i])
        print(f"  system {r} (n={w.n_per[r]}): accel rel-L2 {e:.3e}", flush=True)
        assert e < TOL_ACC
    plan.close()


def test_adjoint_workload_full_size(lib, torch_dev):
    """The adjoint workload at its full size in the benchmark's launch
    configuration (256 systems x 4096 points x 22047 steps, autotuned plan,
    checkpoints every 256 steps stored by the forward pass): the gradient of
    the summed H21-H31 yields for two sampled systems against the oracle's
    own forward, loss gradient and adjoint, and against central differences
    of the GPU forward map along 16 seeded directions (h = 1e-6, bar 1e-5)."""
    from concurrent.futures import ThreadPoolExecutor

    torch, dev = torch_dev
    w = ti.cfg4_adjoint()
    h_lo, h_hi = w.meta["band"]
    a_sc, _ = lib.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    p = lib.make_params(w.dx, w.dt, a_sc, w.nt, mask_fraction=w.mask_frac, mask_power=w.mask_pow)
    plan = lib.Plan(p, w.n_per, adjoint_k=256,
                    options=lib.TDSE_OPT_STORE_CHECKPOINTS | lib.TDSE_OPT_AUTOTUNE)
    E = w.efield(xp={"device": dev}).contiguous()
    k_lo, nk = lib.tdse_harmonic_band(w.nt, w.dt, w.omega, h_lo, h_hi)
    work = torch.empty(2 * w.batch * nk, dtype=torch.float64, device=dev)
    y = torch.empty(w.batch, dtype=torch.float64, device=dev)
    acc = torch.empty_like(E)
    abar = torch.empty_like(E)

    def loss(field):
        lib.tdse_propagate_batch(plan, field, None, acc)
        lib.tdse_harmonic_yield(w.batch, w.nt, w.dt, w.omega, h_lo, h_hi, acc, None, work, y, abar)
        return float(y.sum())

    print(f"adjoint workload full size: {w.batch} x {w.n_per[0]} x {w.nt}, "
          f"layout {plan.layout(w.n_per[0])}", flush=True)
    loss(E)
    grad = torch.empty_like(E)
    st = torch.full((w.batch,), -1, dtype=torch.int32, device=dev)
    lib.tdse_adjoint_batch_stored(plan, plan.checkpoint_generation(), E, abar, grad, st)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    g = grad.cpu().numpy()
    # the oracle side: its own soft-core fit, ground state, forward and loss
    a_ref = oracle_side.soft_core(w.ip, w.dx)
    rows = [0, int(np.argmax(w.e0))]
    e_rows = w.efield(rows=rows)
    with ThreadPoolExecutor(len(rows)) as ex:
        refs = list(ex.map(lambda i: oracle_side.yield_gradient(
            e_rows[i], w.n_per[rows[i]], w.dx, w.dt, a_ref, w.omega, h_lo, h_hi,
            mask_frac=w.mask_frac, mask_pow=w.mask_pow, k=256), range(len(rows))))
    for i, r in enumerate(rows):
        e = rel(g[r], refs[i][1])
        print(f"  system {r}: grad rel-L2 vs oracle {e:.3e}", flush=True)
        assert e < 1e-9
    h = 1e-6
    for d in range(16):
        v = torch.tensor(ti.probe_directions(tuple(E.shape), d), dtype=torch.float64, device=dev)
        fd = (loss(E + h * v) - loss(E - h * v)) / (2 * h)
        ad = float((grad * v).sum())
        print(f"  direction {d}: FD {fd:.10e} adjoint {ad:.10e} rel {abs(fd - ad) / abs(fd):.2e}",
              flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(fd)
    plan.close()


def test_autotuned_plan_matches_oracle(lib, torch_dev):
    """TDSE_OPT_AUTOTUNE: every size gets a timed layout (C in {4, 8, 16},
    systems per workgroup, table placement); results stay within the parity
    bar and agree with the default-layout plan to rounding."""
    torch, dev = torch_dev
    ns = [600, 600, 2048, 3000, 5000]
    dx, dt = 0.2, 0.05
    nt = 150
    efield = 0.06 * np.random.default_rng(12).standard_normal((len(ns), nt + 1))
    print(f"autotune ns={ns} nt={nt}", flush=True)
    plan_t, out_t = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR,
                                 options=lib.TDSE_OPT_AUTOTUNE, want=False)
    plan_d, out_d = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR, want=False)
    for n in sorted(set(ns)):
        lay = plan_t.layout(n)
        info = plan_t.launch_info(n)
        print(f"  n={n}: {lay} {info}", flush=True)
        assert lay.points_per_lane in (4, 8, 16)
        assert lay.lanes % 64 == 0 and lay.lanes * lay.points_per_lane >= n
        assert info.systems_per_workgroup * lay.lanes <= 1024
        assert info.tuned_rate > 0.0
        assert plan_d.launch_info(n).tuned_rate == 0.0
    assert np.all(out_t["status"] == 0)
    for b, n in enumerate(ns):
        ref = oracle_side.propagate(efield[b], n, dx, dt, A_AR, mask_frac=0.1)
        assert rel(out_t["accel"][b], ref["accel"]) < TOL_ACC
        assert rel(out_t["accel"][b], out_d["accel"][b]) < 1e-11
    plan_t.close()
    plan_d.close()


def test_mixed_sizes_share_workgroups(lib, torch_dev):
    """Systems of several sizes and one layout are packed together into
    1024-lane workgroups (with padding subgroups where they do not fill one);
    every system matches the oracle and the packed result equals the
    one-system-per-launch result bitwise."""
    torch, dev = torch_dev
    ns = [2048] * 5 + [2304] * 3 + [3328] * 2 + [600]
    dx, dt = 0.2, 0.05
    nt = 120
    efield = 0.05 * np.random.default_rng(21).standard_normal((len(ns), nt + 1))
    print(f"mixed sizes ns={ns} nt={nt}", flush=True)
    plan, out = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR, want=False)
    _, out_p = _run_forward(lib, torch, dev, ns, efield, dx, dt, A_AR, options=lib.TDSE_OPT_PLAIN,
                            want=False)
    assert np.all(out["status"] == 0)
    assert np.array_equal(out["accel"], out_p["accel"])
    assert np.array_equal(out["psi_final"], out_p["psi_final"])
    for b in (0, 5, 8, 10):
        ref = oracle_side.propagate(efield[b], ns[b], dx, dt, A_AR, mask_frac=0.1)
        assert rel(out["accel"][b], ref["accel"]) < TOL_ACC
    plan.close()
