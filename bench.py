"""Benchmark of the batched 1D-TDSE microscopic step on one MI355X.

Workload (default): the 32 r x 32 z Gaussian-beam focus -- 1024 independent
systems, N = 4096 points (dx = 0.2), dt = 0.05, 20-cycle 800 nm sin^2 pulse,
peak 2e14 W/cm^2 at w0 = 50 um, soft-core argon (Ip = 0.5792), cos^(1/8)
absorber.  Inputs are synthetic and generated on the device.

One timed step = one batched forward solve of the whole batch through
tdse_propagate_batch (graph replay of the persistent kernel): every system
propagated over all Nt steps with the dipole acceleration, <x> and norm
recorded at every sample.  The plan (soft-core fit, tables, ground states)
is built once before the timed region.

Besides the headline `value` (grid-point-steps/s = sum_p N_p Nt / time), the
JSON line carries
  plain       the same kernel launched once per system, serially (subset)
  adjoint     time per gradient of the H21-H31 yield of the 256-system
              adjoint batch (forward + checkpointed reverse sweep)
  roofline    achieved FP64 rate of the forward kernel (52 algorithmic flops
              per grid-point-step) against the 78.6 TFLOP/s vector peak
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
  parity      rel-L2 of the sampled GPU accelerations against that oracle run
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_POINT_STEP = 52.0        # algorithmic FP64 flops per grid-point-step
FP64_VECTOR_PEAK_TFLOPS = 78.6     # 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
HBM_PEAK_GBS = 8000.0              # HBM3E
ADJ_FLOPS_PER_POINT_STEP = 158.0    # forward + recompute + costate step
CSRC = os.path.join(ROOT, "paper_2507_04115_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def source_digest() -> str:
    """sha256 over the kernel sources; HBM counters are valid only for this digest."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def read_traffic(workload: str):
    """HBM bytes per forward launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the same counter's reading
    for a plain device copy of known size).  None when the summary is missing
    or was taken from different kernel sources."""
    path = os.path.join(PROFILES, f"forward_kernel_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest():
        return None
    cb = float(kv["copy_bytes"])
    f_scale = cb / (1024.0 * float(kv["copy_fetch_kib"]))
    w_scale = cb / (1024.0 * float(kv["copy_write_kib"]))
    return 1024.0 * (f_scale * float(kv["fetch_kib_per_dispatch"]) +
                     w_scale * float(kv["write_kib_per_dispatch"]))


def calibrate_copy(mib: int):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_spectrum(torch, L, plan, w, dev, stream):
    """Electron energy distribution of every system of the batch at 256
    energies in [-0.7, 3] a.u. (resolution 0.01), from the plan's ground
    states (the solve costs the same for any state)."""
    n = w.n_per[0]
    gs = torch.empty(2 * n, dtype=torch.float64, device=dev)
    plan.ground_state(n, gs)
    psi = gs.repeat(w.batch).contiguous()
    energies = torch.linspace(-0.7, 3.0, 256, dtype=torch.float64, device=dev)
    spec = torch.empty(w.batch, 256, dtype=torch.float64, device=dev)
    # every (system, energy) solve in flight at once (16 B per point each)
    work = torch.empty(L.tdse_plan_energy_spectrum_work(plan, 256, w.batch * 256) // 8,
                       dtype=torch.float64, device=dev)
    L.tdse_plan_energy_spectrum(plan, psi, energies, 0.01, spec, work)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(3):
        L.tdse_plan_energy_spectrum(plan, psi, energies, 0.01, spec, work)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    solves = float(w.batch * 256)
    del work
    return {"energies": 256, "eps": 0.01, "ms": ms, "solves": solves,
            "grid_point_solves_per_s": solves * n / (ms * 1e-3),
            "hbm_bytes_per_grid_point": 32, "note": "elimination factors per (grid size, energy) "
            "shared by the systems; one lane per (system, energy) carries d' through a "
            "16 B/point workspace (written, then read back)"}


def bench_far_field(torch, L, ti, dev, stream):
    """Far field of the full-volume focus (64 r x 256 z sources) over the
    H25-H35 band of its 1030 nm, 30-cycle pulse, at 64 observation radii,
    from synthetic source spectra (the sum costs the same for any values)."""
    w = ti.cfg5_volume(64, 256)
    k_lo, nk = L.tdse_harmonic_band(w.nt, w.dt, w.omega, 25, 35)
    omega_si = 2 * np.pi * (k_lo + np.arange(nk)) / ((w.nt + 1) * w.dt) / 2.4188843265857e-17
    r = np.unique(w.meta["r_um"]) * 1e-6
    z = np.unique(w.meta["z_um"]) * 1e-6
    wts = np.outer(r * (r[1] - r[0]), np.full(len(z), z[1] - z[0])).ravel()
    g = torch.Generator(device="cpu").manual_seed(7)
    amp = torch.randn(len(r) * len(z), nk, dtype=torch.complex128, generator=g).to(dev)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    geo = (t(r), t(z), t(wts), t(omega_si / 299792458.0))
    ro = t(np.linspace(0.0, 5e-3, 64))
    field = torch.empty(64, nk, dtype=torch.complex128, device=dev)
    amp_bar = torch.empty_like(amp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for adj in (False, True):
        src, dst = (field, amp_bar) if adj else (amp, field)
        L.tdse_far_field(*geo, src, ro, 1.0, dst, adjoint=adj)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(5):
            L.tdse_far_field(*geo, src, ro, 1.0, dst, adjoint=adj)
        e1.record(stream)
        torch.cuda.synchronize()
        res[adj] = e0.elapsed_time(e1) / 5
    terms = float(len(r) * len(z) * nk * 64)
    return {"geometry": f"{len(r)} r x {len(z)} z sources, {nk} bins (H25-H35), 64 observation radii",
            "ms": res[False], "adjoint_ms": res[True], "terms": terms,
            "terms_per_s": terms / (res[False] * 1e-3)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="focus",
                    choices=["focus", "single", "uneven", "uneven-wide", "volume", "sweep"])
    ap.add_argument("--sweep-n", type=int, default=8192, help="grid size of the sweep workload")
    ap.add_argument("--plain-systems", type=int, default=8)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-far-field", action="store_true")
    ap.add_argument("--no-spectrum", action="store_true")
    ap.add_argument("--adjoint-workload", default="adjoint", choices=["adjoint", "volume-axis"],
                    help="256 systems x 4096 points (default) or the 256 on-axis systems of the "
                         "full focal volume (8192 points, 213056 steps)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default lane layouts instead of timing them at plan creation")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the systems are independent; a multi-GPU run would give each GPU its own "
              "plan over a share of them)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import torch

    import tdse_inputs as ti
    from paper_2507_04115_amd import binding as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L.load()

    w = {"focus": ti.cfg2_focus, "single": ti.cfg1_single, "uneven": ti.cfg3_uneven,
         "uneven-wide": lambda: ti.cfg3_uneven(wide=True),
         "volume": ti.cfg5_volume,
         "sweep": lambda: ti.size_sweep(args.sweep_n)}[args.workload]()
    a_sc, e_g = L.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    log(f"workload {w.name}: P={w.batch} nt={w.nt} soft-core a={a_sc:.10f} (E_g={e_g:.13f})")
    p = L.make_params(w.dx, w.dt, a_sc, w.nt, mask_fraction=w.mask_frac, mask_power=w.mask_pow)
    t0 = time.time()
    plan = L.Plan(p, w.n_per, options=0 if args.no_autotune else L.TDSE_OPT_AUTOTUNE)
    layouts = {}
    for n in sorted(set(w.n_per)):
        lay, info = plan.layout(n), plan.launch_info(n)
        layouts[n] = {"points_per_lane": lay.points_per_lane, "lanes": lay.lanes,
                      "scan_levels": lay.scan_levels,
                      "systems_per_workgroup": info.systems_per_workgroup,
                      "lds_tables": info.lds_tables}
    log(f"plan built in {time.time() - t0:.2f} s ({'default layouts' if args.no_autotune else 'autotuned'}); "
        f"{len(layouts)} sizes, first {next(iter(layouts.items()))}")
    E = w.efield(xp={"device": dev}).contiguous()
    acc = torch.empty_like(E)
    xe = torch.empty_like(E)
    nr = torch.empty_like(E)
    status = torch.empty(w.batch, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    point_steps = float(sum(w.n_per)) * w.nt

    for _ in range(args.warmup):
        L.tdse_propagate_batch(plan, E, None, acc, xe, nr, None, status)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        L.tdse_propagate_batch(plan, E, None, acc, xe, nr, None, status)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    value = point_steps / (ms_step * 1e-3)
    st = status.cpu().numpy()
    log(f"batched: {ms_step:.1f} ms/step, {value:.4e} grid-point-steps/s (wall {t_wall:.2f} s); "
        f"status nonzero: {int(np.count_nonzero(st))}")
    achieved = FLOPS_PER_POINT_STEP * value / 1e12

    out = {
        "metric": "TDSE grid-point-steps/s FP64, batched vs plain; adjoint grad time at 1e-9 err",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "systems": w.batch, "grid_points": int(w.n_per[0]) if len(set(w.n_per)) == 1 else "ragged",
                   "nt": w.nt, "dx": w.dx, "dt": w.dt, "grid_point_steps": point_steps,
                   "parallelism": "single-gpu", "autotune": not args.no_autotune,
                   "layout": next(iter(layouts.values())) if len(layouts) == 1 else
                   f"{len(layouts)} sizes"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": read_traffic(w.name),
                     "kernel": "forward_kernel (graph replay incl. counter reset)",
                     "flops_per_grid_point_step": FLOPS_PER_POINT_STEP},
    }

    # ---------------------------------------------------------- plain form
    if not args.no_plain:
        m = min(args.plain_systems, w.batch)
        rows = list(range(m))
        pp = L.Plan(p, [w.n_per[r] for r in rows], options=L.TDSE_OPT_PLAIN)
        Ep = E[:m].contiguous()
        ap_ = torch.empty_like(Ep)
        L.tdse_propagate_batch(pp, Ep, None, ap_)
        torch.cuda.synchronize()
        ev0.record(stream)
        L.tdse_propagate_batch(pp, Ep, None, ap_)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_plain = ev0.elapsed_time(ev1)
        ps_plain = float(sum(w.n_per[r] for r in rows)) * w.nt
        v_plain = ps_plain / (ms_plain * 1e-3)
        same = bool(torch.equal(ap_, acc[:m]))
        out["plain"] = {"value": v_plain, "unit": "grid-point-steps/s", "systems_timed": m,
                        "ms": ms_plain, "batched_over_plain": value / v_plain,
                        "bitwise_equal_to_batched": same}
        log(f"plain: {v_plain:.4e} grid-point-steps/s on {m} systems; batched/plain = {value / v_plain:.1f}")
        pp.close()

    # ------------------------------------------------------------ adjoint
    if not args.no_adjoint:
        wa = ti.cfg4_adjoint() if args.adjoint_workload == "adjoint" else ti.cfg5_axis()
        a_adj = a_sc if wa.dx == w.dx else L.tdse_soft_core_for_ip(wa.ip, 2048, wa.dx, dtau=1.0,
                                                                     tol=1e-13)[0]
        pa = L.make_params(wa.dx, wa.dt, a_adj, wa.nt, mask_fraction=wa.mask_frac,
                           mask_power=wa.mask_pow)
        plan_a = L.Plan(pa, wa.n_per, adjoint_k=256,
                        options=L.TDSE_OPT_STORE_CHECKPOINTS |
                        (0 if args.no_autotune else L.TDSE_OPT_AUTOTUNE))
        lay_a = plan_a.layout(wa.n_per[0])
        Ea = wa.efield(xp={"device": dev}).contiguous()
        acc_a = torch.empty_like(Ea)
        h_lo, h_hi = wa.meta["band"]
        k_lo, nk = L.tdse_harmonic_band(wa.nt, wa.dt, wa.omega, h_lo, h_hi)
        work = torch.empty(2 * wa.batch * max(nk, 1), dtype=torch.float64, device=dev)
        yld = torch.empty(wa.batch, dtype=torch.float64, device=dev)
        abar = torch.empty_like(Ea)
        grad = torch.empty_like(Ea)

        def gradient(stored):
            # forward (stores the checkpoints), loss gradient, reverse sweep; or
            # the adjoint call that runs its own forward pass again
            L.tdse_propagate_batch(plan_a, Ea, None, acc_a)
            L.tdse_harmonic_yield(wa.batch, wa.nt, wa.dt, wa.omega, h_lo, h_hi, acc_a, None, work,
                                  yld, abar)
            if stored:
                L.tdse_adjoint_batch_stored(plan_a, plan_a.checkpoint_generation(), Ea, abar, grad)
            else:
                L.tdse_adjoint_batch(plan_a, Ea, None, abar, grad)

        ms = {}
        for stored in (True, False):
            gradient(stored)
            torch.cuda.synchronize()
            ev0.record(stream)
            gradient(stored)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms[stored] = ev0.elapsed_time(ev1)
        # algorithmic work of one gradient with stored checkpoints: forward,
        # segment recompute and costate step (52 + 52 + 54 flops per
        # grid-point-step); HBM: each recomputed state written to the segment
        # buffer and read back (32 B per grid-point-step) plus the checkpoints
        # written and read once (32 B per grid point every K steps)
        pts_a = float(sum(wa.n_per)) * wa.nt
        t_a = ms[True] * 1e-3
        fl_a = ADJ_FLOPS_PER_POINT_STEP * pts_a / t_a
        by_a = (32.0 + 32.0 / 256) * pts_a / t_a
        out["adjoint"] = {"workload": wa.name, "systems": wa.batch, "nt": wa.nt, "checkpoint_k": 256,
                          "points_per_lane": lay_a.points_per_lane, "lanes": lay_a.lanes,
                          "time_per_gradient_s": ms[True] * 1e-3,
                          "time_per_gradient_recompute_s": ms[False] * 1e-3,
                          "forward_grid_point_steps": float(sum(wa.n_per)) * wa.nt,
                          "loss": f"sum of H{h_lo}-H{h_hi} Hann-windowed yields",
                          "checkpoints": "stored by the forward pass (time_per_gradient_s); "
                                         "recomputed by the adjoint call (..._recompute_s)",
                          "roofline": {"flops_per_grid_point_step": ADJ_FLOPS_PER_POINT_STEP,
                                       "achieved_tflops": fl_a * 1e-12,
                                       "frac_fp64": fl_a * 1e-12 / FP64_VECTOR_PEAK_TFLOPS,
                                       "hbm_bytes_per_grid_point_step": 32.0 + 32.0 / 256,
                                       "achieved_gbs": by_a * 1e-9,
                                       "frac_hbm": by_a * 1e-9 / HBM_PEAK_GBS}}
        log(f"adjoint: {ms[True] * 1e-3:.3f} s per gradient with stored checkpoints, "
            f"{ms[False] * 1e-3:.3f} s recomputing them ({wa.batch} systems)")
        plan_a.close()

    # ------------------------------------------------- energy distribution
    if not args.no_spectrum and len(set(w.n_per)) == 1:
        out["energy_spectrum"] = bench_spectrum(torch, L, plan, w, dev, stream)
        log(f"energy spectrum: {out['energy_spectrum']['ms']:.2f} ms for "
            f"{out['energy_spectrum']['solves']:.0f} (system, energy) solves")

    # ------------------------------------------------------------ far field
    if not args.no_far_field:
        out["far_field"] = bench_far_field(torch, L, ti, dev, stream)
        log(f"far field: {out['far_field']['ms']:.2f} ms, adjoint {out['far_field']['adjoint_ms']:.2f} ms "
            f"({out['far_field']['terms']:.3g} source-observation-frequency terms)")

    # ------------------------------------------------------- CPU baseline
    if not args.no_cpu:
        import oracle

        nth = args.cpu_threads or min(16, os.cpu_count() or 1)
        # a stratified sample: rows spread over the batch (two per thread),
        # plus the smallest and the largest grid
        by_n = np.argsort(np.asarray(w.n_per), kind="stable")
        rows = np.array(sorted(set(np.linspace(0, w.batch - 1, 2 * nth).round().astype(int).tolist())
                               | {int(by_n[0]), int(by_n[-1])}))
        # the oracle's own soft-core fit and ground states (outside the timing)
        a_ref = oracle.soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0)[0]
        gs = {}
        psi_list = []
        for r in rows:
            n = w.n_per[r]
            if n not in gs:
                gs[n] = oracle.ground_state(n, w.dx, a_ref, dtau=1.0, tol=1e-14)[0]
            psi_list.append(gs[n])
        e_rows = np.ascontiguousarray(w.efield(rows=rows))
        t0 = time.perf_counter()
        ref = oracle.propagate_batch(e_rows, psi_list, w.dx, w.dt, a_ref, mask_frac=w.mask_frac,
                                     mask_pow=w.mask_pow, nthreads=nth)
        t_cpu = time.perf_counter() - t0
        ps_cpu = float(sum(w.n_per[r] for r in rows)) * w.nt
        # one core: the first sampled system alone
        t1 = time.perf_counter()
        oracle.propagate_batch(e_rows[:1], psi_list[:1], w.dx, w.dt, a_ref, mask_frac=w.mask_frac,
                               mask_pow=w.mask_pow, nthreads=1)
        t1 = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": ps_cpu / t_cpu, "unit": "grid-point-steps/s", "cores": nth,
                               "kind": "oracle",
                               "sample": f"{len(rows)} systems of the same batch (rows spread over it, "
                                         f"smallest and largest grid included), full {w.nt} steps, "
                                         f"one system per thread at a time on {nth} threads, {t_cpu:.1f} s",
                               "single_core_value": float(w.n_per[rows[0]]) * w.nt / t1,
                               "cpu_model": cpu_model()}
        got = acc[torch.as_tensor(rows, device=dev)].cpu().numpy()
        errs = [float(np.linalg.norm(got[i] - ref["accel"][i]) / np.linalg.norm(ref["accel"][i]))
                for i in range(len(rows))]
        out["parity"] = {"accel_rel_l2_max": max(errs), "systems_checked": len(rows),
                         "tolerance": 1e-9}
        log(f"cpu oracle: {ps_cpu / t_cpu:.3e} grid-point-steps/s on {nth} threads "
            f"({out['cpu_baseline']['single_core_value']:.3e} on one core, {cpu_model()}); "
            f"parity max rel-L2 {max(errs):.2e} over {len(rows)} systems")

    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
