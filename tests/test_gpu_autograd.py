"""torch.autograd path (paper_2507_04115_amd.autograd) on the GPU: the
gradient of a harmonic-yield loss through TDSEFunction / HarmonicYield
against the CPU oracle's adjoint of the same loss (the oracle's own forward,
ground state and loss gradient) and against central differences of the GPU
forward map (bar: 1e-5 relative)."""
import numpy as np
import pytest

import oracle_side
import tdse_inputs as ti

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def setup(lib):
    import torch

    from paper_2507_04115_amd import autograd as AG

    dev = torch.device("cuda:0")
    ns = [256, 320, 256]
    dx, dt, a = 0.4, 0.05, 1.1
    om, nc = 0.25, 3
    nt = ti.n_steps(om, nc, dt)
    efield = ti.sin2_pulse(np.array([0.1, 0.08, 0.12]), om, nc, dt, nt=nt)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    batch = AG.TDSEBatch(p, ns, adjoint_k=64)
    yield dict(torch=torch, dev=dev, AG=AG, ns=ns, dx=dx, dt=dt, a=a, om=om, nt=nt,
               efield=efield, batch=batch)
    batch.close()


def test_yield_gradient_matches_oracle_adjoint(setup, lib):
    s = setup
    torch, AG = s["torch"], s["AG"]
    print(f"autograd yield gradient ns={s['ns']} nt={s['nt']}", flush=True)
    E = torch.tensor(s["efield"], dtype=torch.float64, device=s["dev"], requires_grad=True)
    acc = s["batch"](E)
    w = torch.tensor([1.0, 0.5, 2.0], dtype=torch.float64, device=s["dev"])
    y = AG.HarmonicYield.apply(acc, s["dt"], s["om"], 3, 9)
    (w * y).sum().backward()
    g = E.grad.cpu().numpy()
    yv = y.detach().cpu().numpy()
    for b in range(3):
        y_ref, g_ref = oracle_side.yield_gradient(s["efield"][b], s["ns"][b], s["dx"], s["dt"],
                                                  s["a"], s["om"], 3, 9, weight=float(w[b]),
                                                  mask_frac=0.2, k=64)
        r = rel(g[b], g_ref)
        print(f"  system {b}: yield rel err {abs(yv[b] - y_ref) / y_ref:.3e}, "
              f"grad rel-L2 vs oracle adjoint {r:.3e}", flush=True)
        assert abs(yv[b] - y_ref) <= 1e-9 * y_ref
        assert r < 1e-9


def test_gradient_matches_central_differences_of_gpu_forward(setup, lib):
    s = setup
    torch, AG = s["torch"], s["AG"]
    E = torch.tensor(s["efield"], dtype=torch.float64, device=s["dev"], requires_grad=True)
    loss = AG.HarmonicYield.apply(s["batch"](E), s["dt"], s["om"], 3, 9).sum()
    loss.backward()
    g = E.grad.detach()
    h = 1e-6
    for d in range(2):
        v = torch.tensor(ti.probe_directions(E.shape, d), dtype=torch.float64, device=s["dev"])
        with torch.no_grad():
            lp = AG.HarmonicYield.apply(s["batch"](E + h * v), s["dt"], s["om"], 3, 9).sum()
            lm = AG.HarmonicYield.apply(s["batch"](E - h * v), s["dt"], s["om"], 3, 9).sum()
        fd = float((lp - lm) / (2 * h))
        ad = float((g * v).sum())
        print(f"  direction {d}: FD {fd:.10e} adjoint {ad:.10e}", flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(fd)


def test_torch_side_loss_chains_through_adjoint(setup, lib):
    """A loss written with torch ops on the acceleration: accel_bar comes from
    torch autograd, the rest from the adjoint kernel."""
    s = setup
    torch = s["torch"]
    E = torch.tensor(s["efield"], dtype=torch.float64, device=s["dev"], requires_grad=True)
    acc = s["batch"](E)
    (0.5 * (acc ** 2).sum()).backward()
    g = E.grad.cpu().numpy()
    for b in (0, 2):
        # the same loss on the oracle: accel_bar = its own acceleration
        n = s["ns"][b]
        acc_ref = oracle_side.propagate(s["efield"][b], n, s["dx"], s["dt"], s["a"],
                                        mask_frac=0.2)["accel"]
        g_ref, _ = oracle_side.adjoint(s["efield"][b], acc_ref, n, s["dx"], s["dt"], s["a"],
                                       mask_frac=0.2, k=64)
        r = rel(g[b], g_ref)
        print(f"  system {b}: grad rel-L2 (torch loss) {r:.3e}", flush=True)
        assert r < 1e-9


def test_stored_checkpoints_through_autograd(setup, lib):
    """Two forwards, then the two backwards in reverse order through a plan
    that stores checkpoints: the second forward's backward reads the store,
    the first one's finds it rewritten and recomputes; both equal the
    gradients of the plan that always recomputes."""
    s = setup
    torch, AG = s["torch"], s["AG"]
    p = lib.make_params(s["dx"], s["dt"], s["a"], s["nt"], mask_fraction=0.2)
    sb = AG.TDSEBatch(p, s["ns"], adjoint_k=64, store_checkpoints=True)
    grads = {}
    for name, batch in (("stored", sb), ("recompute", s["batch"])):
        E1 = torch.tensor(s["efield"], dtype=torch.float64, device=s["dev"], requires_grad=True)
        E2 = torch.tensor(1.1 * s["efield"], dtype=torch.float64, device=s["dev"],
                          requires_grad=True)
        y1 = AG.HarmonicYield.apply(batch(E1), s["dt"], s["om"], 3, 9).sum()
        y2 = AG.HarmonicYield.apply(batch(E2), s["dt"], s["om"], 3, 9).sum()
        y2.backward()
        y1.backward()
        grads[name] = (E1.grad.cpu().numpy(), E2.grad.cpu().numpy())
    for a_, b_ in zip(grads["stored"], grads["recompute"]):
        assert np.array_equal(a_, b_)
    sb.close()


def test_spectral_phase_gradient_of_on_axis_yield(lib):
    """The full-volume workload's optimisation problem, small: the harmonic
    yield summed over the on-axis points of a 2 r x 3 z focus, as a function
    of 64 spectral-phase coefficients of the driver.  dl/dc comes from
    autograd through the FFT map, TDSEFunction's adjoint (off-axis rows have
    an all-zero accel_bar and are skipped) and HarmonicYield; it must match
    central differences of the GPU forward map (bar: 1e-5 relative)."""
    import torch

    from paper_2507_04115_amd import autograd as AG
    from paper_2507_04115_amd.driver import SpectralPhase

    dev = torch.device("cuda:0")
    om, nc, dt, dx, a = 0.25, 3, 0.05, 0.4, 1.1
    nt = ti.n_steps(om, nc, dt)
    nr, nz = 2, 3
    e0, ph, r, _ = ti.gaussian_focus(nr, nz, 50.0, 800.0, 2e14)
    E0 = torch.tensor(ti.sin2_pulse(e0, om, nc, dt, phase=ph, nt=nt), dtype=torch.float64,
                      device=dev)
    p = lib.make_params(dx, dt, a, nt, mask_fraction=0.2)
    batch = AG.TDSEBatch(p, [256] * (nr * nz), adjoint_k=64, store_checkpoints=True)
    sp = SpectralPhase(E0, 64)
    on_axis = torch.tensor((r == 0.0).astype(np.float64), device=dev)
    print(f"spectral phase: {nr}x{nz} focus, nt={nt}, band bins {sp.band}", flush=True)

    def loss(c):
        return (AG.HarmonicYield.apply(batch(sp(c)), dt, om, 3, 9) * on_axis).sum()

    c = torch.tensor(np.random.default_rng(5).normal(0.0, 0.3, 64), dtype=torch.float64,
                     device=dev, requires_grad=True)
    loss(c).backward()
    g = c.grad.detach()
    assert torch.count_nonzero(g) > 0
    h = 1e-6
    for d in range(2):
        v = torch.tensor(np.random.default_rng(20 + d).standard_normal(64), dtype=torch.float64,
                         device=dev)
        with torch.no_grad():
            fd = float((loss(c + h * v) - loss(c - h * v)) / (2 * h))
        ad = float((g * v).sum())
        print(f"  direction {d}: FD {fd:.10e} adjoint {ad:.10e}", flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(fd)
    batch.close()


def test_backward_without_adjoint_plan_raises(lib):
    import torch

    from paper_2507_04115_amd import autograd as AG

    p = lib.make_params(0.4, 0.05, 1.1, 20, mask_fraction=0.2)
    plan = lib.Plan(p, [256])
    E = torch.zeros(1, 21, dtype=torch.float64, device="cuda:0", requires_grad=True)
    acc = AG.TDSEFunction.apply(E, plan)
    with pytest.raises(RuntimeError):
        acc.sum().backward()
    plan.close()
