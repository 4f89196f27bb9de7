"""Per-step populations (tdse_propagate_batch_populations): the ground-state
population |dx <phi, psi(t)>|^2 and the volumetric population near the
nucleus at every sample, reduced in the time loop, against the oracle's
populations of its own states stepped one at a time.  The dipole outputs of
the same call equal tdse_propagate_batch's bitwise."""
import numpy as np
import pytest

import oracle
import oracle_side
import tdse_inputs as ti

pytestmark = pytest.mark.gpu
A_AR = 1.1891671


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _oracle_populations(efield_row, psi0, phi, dx, dt, a, radius, mask_frac):
    psi = np.asarray(psi0, np.complex128).copy()
    gs, vol = [], []
    for i in range(len(efield_row)):
        g, v = oracle.populations(psi, phi, dx, radius)
        gs.append(g)
        vol.append(v)
        if i + 1 < len(efield_row):
            psi = oracle.step(psi, dx, dt, a, 1.0, efield_row[i], mask_frac=mask_frac)
    return np.array(gs), np.array(vol)


@pytest.mark.parametrize("options,ref_kind", [(0, "plan"), (0, "given"), ("plain", "plan")])
def test_populations_every_sample_match_oracle(lib, options, ref_kind):
    import torch

    dev = torch.device("cuda:0")
    ns = [300, 512, 1030, 2100, 9000]
    # 161 steps: both the 16-step blocks of the populations variant and the
    # 32-step blocks of the plain one end with a one-step block
    dx, dt, nt, radius = 0.2, 0.05, 161, 6.0
    rng = np.random.default_rng(77)
    om = 0.057
    efield = ti.sin2_pulse(np.linspace(0.05, 0.12, len(ns)), om, 1, dt, nt=nt)
    efield = np.ascontiguousarray(efield + 0.02 * rng.standard_normal(efield.shape))
    p = lib.make_params(dx, dt, A_AR, nt, mask_fraction=0.1)
    opt = lib.TDSE_OPT_PLAIN if options == "plain" else options
    plan = lib.Plan(p, ns, options=opt)
    off = plan.psi_offsets()
    E = torch.tensor(efield, device=dev)
    acc = torch.empty_like(E)
    nr = torch.empty_like(E)
    gsp = torch.full_like(E, np.nan)
    vol = torch.full_like(E, np.nan)
    st = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
    refs = None
    psi_ref = None
    if ref_kind == "given":
        refs = [ti.random_state(n, 300 + b, width=min(8.0, n * dx / 8), k0=0.4, dx=dx)
                for b, n in enumerate(ns)]
        psi_ref = torch.tensor(np.concatenate(refs), dtype=torch.complex128, device=dev)
    lib.tdse_propagate_batch_populations(plan, E, None, acc, radius, gs_pop=gsp, vol_pop=vol,
                                         norm=nr, sys_status=st, psi_ref=psi_ref)
    acc_plain = torch.empty_like(E)
    lib.tdse_propagate_batch(plan, E, None, acc_plain)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    assert torch.equal(acc, acc_plain)
    gsp, vol, nr = gsp.cpu().numpy(), vol.cpu().numpy(), nr.cpu().numpy()
    print(f"populations options={options} ref={ref_kind}: layouts "
          f"{[plan.layout(n).points_per_lane for n in ns]}", flush=True)
    for b, n in enumerate(ns):
        psi0 = oracle_side.ground_state(n, dx, A_AR)
        phi = psi0 if refs is None else refs[b]
        g_ref, v_ref = _oracle_populations(efield[b], psi0, phi, dx, dt, A_AR, radius, 0.1)
        eg, ev = rel(gsp[b], g_ref), rel(vol[b], v_ref)
        print(f"  n={n}: gs pop rel-L2 {eg:.2e} (from {gsp[b][0]:.6f} to {gsp[b][-1]:.6f}), "
              f"vol pop {ev:.2e}", flush=True)
        assert eg < 1e-9 and ev < 1e-9
        assert np.all(vol[b] <= nr[b] * (1 + 1e-12))
        if refs is None:
            assert abs(gsp[b][0] - 1.0) < 1e-10      # starts in the ground state
    plan.close()


def test_populations_refused_on_storing_plans_and_without_outputs(lib):
    import torch

    dev = torch.device("cuda:0")
    p = lib.make_params(0.2, 0.05, A_AR, 20)
    E = torch.zeros(1, 21, dtype=torch.float64, device=dev)
    acc = torch.empty_like(E)
    g = torch.empty_like(E)
    store = lib.Plan(p, [256], adjoint_k=8, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    with pytest.raises(lib.TDSEError) as ei:
        lib.tdse_propagate_batch_populations(store, E, None, acc, 5.0, gs_pop=g)
    assert ei.value.status == lib.TDSE_E_UNSUPPORTED
    plan = lib.Plan(p, [256])
    with pytest.raises(lib.TDSEError) as ei:
        lib.tdse_propagate_batch_populations(plan, E, None, acc, 5.0)
    assert ei.value.status == lib.TDSE_E_INVALID
    with pytest.raises(ValueError):
        lib.tdse_propagate_batch_populations(plan, E, None, acc, 5.0, gs_pop=g[:, :10])
    store.close()
    plan.close()
