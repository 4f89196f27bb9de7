"""Full-length GPU parity on the longest and largest configurations, in the
benchmark's launch configuration (autotuned plans; the focal volume split
into the benchmark's 20 time segments chained through psi_final -> psi0):

* the full focal volume (N = 8192, dx = 0.15, dt = 0.02, 213 056 steps):
  three systems -- the hottest on-axis point, an off-axis point and the
  weakest corner -- against the oracle over the whole pulse, and the
  gradient of the on-axis H25-H35 yield against central differences;
* the largest grid of the wide uneven batch (N = 16 384, 16 points per lane)
  and the 12-point layout (N = 12 288) over the full 85 924 steps.

The oracle side starts from its own soft-core fit and ground states; the
oracle runs one system per host thread."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import bench
import oracle_side
import tdse_inputs as ti

pytestmark = pytest.mark.gpu
TOL_ACC = 1e-9


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _oracle_rows(w, rows, a_ref):
    """The oracle's accelerations of `rows` over the whole pulse, one thread each."""
    e_rows = w.efield(rows=rows)
    with ThreadPoolExecutor(len(rows)) as ex:
        return list(ex.map(lambda i: oracle_side.propagate(
            e_rows[i], w.n_per[rows[i]], w.dx, w.dt, a_ref, mask_frac=w.mask_frac,
            mask_pow=w.mask_pow)["accel"], range(len(rows))))


def test_segmented_solve_equals_single_solve(lib):
    """A solve split into time segments (each continuing from the previous
    segment's psi_final) gives the single solve's outputs to rounding, and
    both match the oracle."""
    import torch

    dev = torch.device("cuda:0")
    ns = [512, 700, 1024, 3000]
    w = ti.Workload("segments", 0.2, 0.05, 0.057, 2, 600, ns,
                    np.array([0.05, 0.06, 0.07, 0.08]), np.array([0.0, 0.3, 0.6, 0.9]))
    a = 1.1891671
    single = bench.SegmentedSolve(torch, lib, w, a, 1, 0, dev)
    seg = bench.SegmentedSolve(torch, lib, w, a, 7, 0, dev)
    assert seg.nseg == 7 and sum(seg.lens) == w.nt and single.nseg == 1
    single.run(0)
    for c in range(seg.nseg):
        seg.run(c)
    torch.cuda.synchronize()
    assert single.statuses_clean() and seg.statuses_clean()
    rows = list(range(len(ns)))
    s1, s7 = single.series(rows), seg.series(rows)
    assert s1.shape == s7.shape == (len(ns), w.nt + 1)
    e_rows = w.efield()
    for b, n in enumerate(ns):
        r_seg = rel(s7[b], s1[b])
        ref = oracle_side.propagate(e_rows[b], n, w.dx, w.dt, a, mask_frac=w.mask_frac)["accel"]
        print(f"  n={n}: segmented vs single {r_seg:.2e}, vs oracle {rel(s7[b], ref):.2e}",
              flush=True)
        assert r_seg < 1e-12
        assert rel(s7[b], ref) < TOL_ACC and rel(s1[b], ref) < TOL_ACC
    single.close()
    seg.close()


def _volume_picks(w):
    r, z = w.meta["r_um"], w.meta["z_um"]
    hot = int(np.argmax(w.e0))
    rs = np.unique(r)
    off = int(np.argmin(np.abs(r - rs[len(rs) // 3]) * 1e6 + np.abs(z - z[hot])))
    weak = int(np.argmin(w.e0))
    return [hot, off, weak]


def test_volume_full_length_sampled(lib):
    """Full focal volume, whole 213 056-step pulse, benchmark launch
    configuration (autotuned, 20 chained time segments), on a 512-system
    sub-batch spread over the volume: the hottest on-axis system, an
    off-axis one and the weakest corner against the oracle."""
    import torch

    dev = torch.device("cuda:0")
    w = ti.cfg5_volume()
    picks = _volume_picks(w)
    rows = sorted(set(np.linspace(0, w.batch - 1, 512 - len(picks)).round().astype(int).tolist())
                  | set(picks))
    sw = w.subset(rows)
    a_sc, _ = lib.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    print(f"volume sub-batch {sw.batch} x {w.n_per[0]} x {w.nt}, picks {picks} "
          f"(r {[float(w.meta['r_um'][p]) for p in picks]} um)", flush=True)
    solve = bench.SegmentedSolve(torch, lib, sw, a_sc, 20, lib.TDSE_OPT_AUTOTUNE, dev)
    print(f"  layout {bench.kernel_shape(solve.plan(), w.n_per[0])}", flush=True)
    for c in range(solve.nseg):
        solve.run(c)
    torch.cuda.synchronize()
    assert solve.statuses_clean()
    got = solve.series([rows.index(p) for p in picks])
    a_ref = oracle_side.soft_core(w.ip, w.dx)
    refs = _oracle_rows(w, picks, a_ref)
    for i, p in enumerate(picks):
        e = rel(got[i], refs[i])
        print(f"  system {p} (E0 {w.e0[p]:.4f}): accel rel-L2 {e:.3e}", flush=True)
        assert e < TOL_ACC
    solve.close()


def test_volume_axis_adjoint_matches_finite_differences(lib):
    """Gradient of the summed on-axis H25-H35 yields over the whole pulse of
    the focal volume (8 on-axis systems around the focus, K = 256, stored
    checkpoints, autotuned as the benchmark's on-axis adjoint) against
    central differences of the GPU forward map along two seeded directions
    (h = 1e-6, bar 1e-5)."""
    import torch

    dev = torch.device("cuda:0")
    wa = ti.cfg5_axis()
    hot = int(np.argmax(wa.e0))
    sw = wa.subset(list(range(hot - 4, hot + 4)))
    h_lo, h_hi = wa.meta["band"]
    a_sc, _ = lib.tdse_soft_core_for_ip(wa.ip, 2048, wa.dx, dtau=1.0, tol=1e-13)
    p = lib.make_params(sw.dx, sw.dt, a_sc, sw.nt, mask_fraction=sw.mask_frac,
                        mask_power=sw.mask_pow)
    plan = lib.Plan(p, sw.n_per, adjoint_k=256,
                    options=lib.TDSE_OPT_STORE_CHECKPOINTS | lib.TDSE_OPT_AUTOTUNE)
    fwd = lib.Plan(p, sw.n_per, options=lib.TDSE_OPT_AUTOTUNE)
    E = sw.efield(xp={"device": dev}).contiguous()
    k_lo, nk = lib.tdse_harmonic_band(sw.nt, sw.dt, sw.omega, h_lo, h_hi)
    work = torch.empty(2 * sw.batch * nk, dtype=torch.float64, device=dev)
    y = torch.empty(sw.batch, dtype=torch.float64, device=dev)
    acc = torch.empty_like(E)
    abar = torch.empty_like(E)
    print(f"on-axis adjoint: {sw.batch} x {sw.n_per[0]} x {sw.nt}, layout "
          f"{plan.layout(sw.n_per[0])}", flush=True)

    def loss(pl, field, want_abar=False):
        lib.tdse_propagate_batch(pl, field, None, acc)
        lib.tdse_harmonic_yield(sw.batch, sw.nt, sw.dt, sw.omega, h_lo, h_hi, acc, None, work, y,
                                abar if want_abar else None)
        return float(y.sum())

    l0 = loss(plan, E, True)
    grad = torch.empty_like(E)
    st = torch.full((sw.batch,), -1, dtype=torch.int32, device=dev)
    lib.tdse_adjoint_batch_stored(plan, plan.checkpoint_generation(), E, abar, grad, st)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    assert abs(loss(fwd, E) - l0) <= 1e-10 * abs(l0)
    h = 1e-6
    for d in range(2):
        v = torch.tensor(ti.probe_directions(tuple(E.shape), d), dtype=torch.float64, device=dev)
        fd = (loss(fwd, E + h * v) - loss(fwd, E - h * v)) / (2 * h)
        ad = float((grad * v).sum())
        print(f"  direction {d}: FD {fd:.10e} adjoint {ad:.10e} rel {abs(fd - ad) / abs(fd):.2e}",
              flush=True)
        assert abs(fd - ad) <= 1e-5 * abs(fd)
    plan.close()
    fwd.close()


def test_uneven_wide_largest_grid_and_twelve_points_full_length(lib, monkeypatch):
    """The wide uneven batch over its full 85 924 steps: the largest grid
    (N = 16 384, 16 points per lane) in an autotuned plan over the batch's
    largest systems, and N = 12 288 in the forward-only 12-point layout
    (forced), each against the oracle."""
    import torch

    dev = torch.device("cuda:0")
    w = ti.cfg3_uneven(wide=True)
    ns = np.asarray(w.n_per)
    big = [int(i) for i in np.nonzero(ns == 16384)[0][:8]]
    twelve = [int(i) for i in np.nonzero(ns == 12288)[0][:8]]
    sw = w.subset(big + twelve)
    a_sc, _ = lib.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    solve = bench.SegmentedSolve(torch, lib, sw, a_sc, 1, lib.TDSE_OPT_AUTOTUNE, dev)
    lay = {n: solve.plan().layout(n).points_per_lane for n in (16384, 12288)}
    print(f"uneven-wide sub-batch {sw.batch} systems, nt={w.nt}, autotuned layouts {lay}",
          flush=True)
    assert lay[16384] == 16
    solve.run(0)
    # the 12-point layout, forced, on the N = 12 288 systems alone
    tw = w.subset(twelve)
    monkeypatch.setenv("TDSE_LAYOUT_C", "12")
    forced = bench.SegmentedSolve(torch, lib, tw, a_sc, 1, 0, dev)
    p_adj = lib.make_params(w.dx, w.dt, a_sc, 10)
    with pytest.raises(lib.TDSEError) as ei:
        lib.Plan(p_adj, [12288], adjoint_k=4)
    monkeypatch.delenv("TDSE_LAYOUT_C")
    assert "forward-only" in str(ei.value)
    assert forced.plan().layout(12288).points_per_lane == 12
    forced.run(0)
    torch.cuda.synchronize()
    assert solve.statuses_clean() and forced.statuses_clean()
    a_ref = oracle_side.soft_core(w.ip, w.dx)
    picks = [big[0], twelve[0]]
    refs = _oracle_rows(w, picks, a_ref)
    got_big = solve.series([0])[0]
    got_12 = forced.series([0])[0]
    got_12_auto = solve.series([len(big)])[0]
    for name, got, ref in [("16384 (C=16)", got_big, refs[0]), ("12288 (C=12)", got_12, refs[1]),
                           (f"12288 (autotuned C={lay[12288]})", got_12_auto, refs[1])]:
        e = rel(got, ref)
        print(f"  n={name}: accel rel-L2 {e:.3e}", flush=True)
        assert e < TOL_ACC
    solve.close()
    forced.close()
