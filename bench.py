"""Benchmark of the batched 1D-TDSE microscopic step on one MI355X.

Workload (default): the full focal volume -- 16 384 independent systems on a
64 r x 256 z Gaussian-beam grid (w0 = 80 um, 1030 nm, 2.5e14 W/cm^2,
30-cycle sin^2), N = 8192 points (dx = 0.15), dt = 0.02, 213 056 steps,
soft-core argon (Ip = 0.5792), cos^(1/8) absorber on the outer tenth of the
grid at each side.  Inputs are synthetic and generated on the device before
the timed region.

The time loop of that solve is split into as many segments as there are
timed steps; one timed step propagates every system through one segment
(tdse_propagate_batch, graph replay of the persistent kernel, starting from
the previous segment's psi_final), so the K timed steps are exactly one full
solve of the volume.  The dipole acceleration, <x> and the norm are recorded
at every sample.  The warm-up steps run the first segments of the same solve.
The plans (soft-core fit, tables, ground states, autotuned layout) are built
once before the timed region.  --workload focus (or any other) times whole
solves instead (one step = one solve).

Besides the headline `value` (grid-point-steps/s = sum_p N_p Nt / time), the
JSON line carries
  roofline      achieved FP64 rate of the forward kernel (52 algorithmic flops
                per grid-point-step) against the 78.6 TFLOP/s vector peak,
                its LDS traffic against the LDS peak, and its occupancy
  plain         the same kernel launched once per system, serially (subset)
  focus         the 1024-system focus batch (N = 4096, 44 093 steps)
  adjoint       time per gradient of the H21-H31 yield of the 256-system
                adjoint batch (forward + checkpointed reverse sweep)
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
  parity        rel-L2 of the sampled GPU accelerations against that oracle run
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
# LDS read bandwidth: 256 CUs x 128 B/clk x 2.4 GHz
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12
ADJ_FLOPS_PER_POINT_STEP = 158.0    # forward + recompute + costate step
CSRC = os.path.join(ROOT, "paper_2507_04115_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


# the translation unit of the forward kernel and the headers it includes:
# the HBM counters describe that kernel only
FORWARD_SOURCES = ("tdse_forward.hip", "tdse_device.hpp", "tdse_internal.hpp", "tdse_kernels.hpp")


def source_digest() -> str:
    """sha256 over the forward kernel's sources; HBM counters are valid only for this digest."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(FORWARD_SOURCES):
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
    # every (system, energy) solve in flight at once (2 B per point each)
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
    # algorithmic HBM bytes: psi in (16 B per point and system), the shared
    # factors (48 B per point and energy), the spectrum out; plus the d'
    # group starts the kernel keeps (1 B per point and solve, written and
    # read back)
    algo = 16.0 * n * w.batch + 48.0 * n * 256 + 8.0 * solves
    ckpt = 2.0 * 1.0 * n * solves
    return {"energies": 256, "eps": 0.01, "ms": ms, "solves": solves,
            "grid_point_solves_per_s": solves * n / (ms * 1e-3),
            "algorithmic_hbm_bytes": algo, "group_start_bytes": ckpt,
            "hbm_gbs_incl_group_starts": (algo + ckpt) / (ms * 1e-3) / 1e9,
            "note": "elimination factors per (grid size, energy) shared by the systems, "
                    "read as scalar loads; one lane per (system, energy), one energy and 64 "
                    "systems of one size per wavefront, M2 psi point-interleaved per size; "
                    "d' kept in registers in groups of 16 points, recomputed from each "
                    "group's start value in the backward sweep"}


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


def cpu_model() -> dict:
    """Host CPU model and sizes (lscpu's model name, sockets, cores, threads)."""
    info = {"model": "unknown"}
    try:
        import subprocess

        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name", "unknown")
        for key, name in (("Socket(s)", "sockets"), ("Core(s) per socket", "cores_per_socket"),
                          ("Thread(s) per core", "threads_per_core"), ("CPU(s)", "cpus")):
            if key in kv:
                info[name] = int(kv[key])
        # the rest of lscpu's identification (the model name alone can be generic)
        for key, name in (("Vendor ID", "vendor"), ("CPU family", "family"), ("Model", "model_id"),
                          ("Stepping", "stepping"), ("CPU max MHz", "max_mhz"),
                          ("L3 cache", "l3_cache"), ("Hypervisor vendor", "hypervisor"),
                          ("Architecture", "arch")):
            if key in kv:
                info[name] = kv[key]
    except Exception:
        pass
    try:
        info["threads_available"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["threads_available"] = os.cpu_count() or 1
    return info


def adjoint_cpu_leg(wa, g_gpu, h_lo, h_hi, cpu_threads=0) -> dict:
    """The oracle's gradient of the same loss for a bounded sample of the
    adjoint workload's systems, one system per thread, each from the
    oracle's own soft-core fit, ground state, forward pass and loss gradient
    (no value of the GPU path goes in), timed, and compared with the GPU
    gradient rows of those systems."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    cpu = cpu_model()
    nth = cpu_threads or max(1, min(16, cpu["threads_available"]))
    rows = sorted({int(np.argmax(wa.e0))} |
                  set(np.linspace(0, wa.batch - 1, nth).round().astype(int).tolist()))[:nth]
    n = wa.n_per[0]
    a_ref = oracle.soft_core_for_ip(wa.ip, 2048, wa.dx, dtau=1.0)[0]
    psi0 = oracle.ground_state(n, wa.dx, a_ref, dtau=1.0, tol=1e-14)[0]
    e_rows = np.ascontiguousarray(wa.efield(rows=rows))
    kw = dict(mask_frac=wa.mask_frac, mask_pow=wa.mask_pow)

    def one(i):
        accel = oracle.propagate(e_rows[i], psi0, wa.dx, wa.dt, a_ref, **kw)["accel"]
        _, ab = oracle.harmonic_yield(accel[None, :], wa.dt, wa.omega, h_lo, h_hi)
        g, _ = oracle.adjoint(e_rows[i], psi0, ab[0], wa.dx, wa.dt, a_ref, k=256, **kw)
        return g

    t0 = time.perf_counter()
    with ThreadPoolExecutor(nth) as ex:
        gs = list(ex.map(one, range(len(rows))))
    t = time.perf_counter() - t0
    errs = [float(np.linalg.norm(g_gpu[r] - gs[i]) / np.linalg.norm(gs[i])) for i, r in enumerate(rows)]
    return {"cpu_baseline": {"kind": "oracle", "systems": len(rows), "cores": nth, "seconds": t,
                             "time_per_gradient_s_extrapolated": t * wa.batch / len(rows),
                             "extrapolation": "linear in the number of systems (one per thread)",
                             "sample": f"{len(rows)} systems of the batch (the hottest and the rest "
                                       f"spread over it), whole pulse ({wa.nt} steps): forward, "
                                       f"loss gradient and adjoint each, one system per thread"},
            "parity": {"grad_rel_l2_max": max(errs), "systems_checked": len(rows),
                       "tolerance": 1e-9,
                       "oracle_side": "own soft-core fit, ground state, forward and loss gradient"}}


def seg_lengths(nt: int, nseg: int):
    """Lengths of nseg consecutive time segments covering nt steps."""
    nseg = max(1, min(nseg, nt)) if nt > 0 else 1
    base, extra = divmod(nt, nseg)
    return [base + 1] * extra + [base] * (nseg - extra)


class SegmentedSolve:
    """One solve of a workload split into time segments: segment c propagates
    every system over steps [start_c, start_c + len_c], continuing from the
    previous segment's final states (psi_final -> psi0).  One plan per
    distinct segment length (at most two)."""

    def __init__(self, torch, L, w, a_sc, nseg, options, dev):
        self.torch, self.L, self.w, self.dev = torch, L, w, dev
        self.lens = seg_lengths(w.nt, nseg)
        self.starts = [0]
        for n in self.lens[:-1]:
            self.starts.append(self.starts[-1] + n)
        self.plans = {}
        for n in sorted(set(self.lens), reverse=True):
            p = L.make_params(w.dx, w.dt, a_sc, n, mask_fraction=w.mask_frac, mask_power=w.mask_pow)
            self.plans[n] = L.Plan(p, w.n_per, options=options)
        self.E, self.acc, self.xe, self.nr, self.st = [], [], [], [], []
        for i0, n in zip(self.starts, self.lens):
            e = w.efield(xp={"device": dev}, i0=i0, nt=n).contiguous()
            self.E.append(e)
            self.acc.append(torch.empty_like(e))
            self.xe.append(torch.empty_like(e))
            self.nr.append(torch.empty_like(e))
            self.st.append(torch.full((w.batch,), -1, dtype=torch.int32, device=dev))
        npsi = 2 * int(sum(w.n_per))
        self.psi = [torch.empty(npsi, dtype=torch.float64, device=dev) if len(self.lens) > 1 else None
                    for _ in range(2)]
        self.work = [float(sum(w.n_per)) * n for n in self.lens]

    @property
    def nseg(self):
        return len(self.lens)

    def plan(self, c=0):
        return self.plans[self.lens[c]]

    def run(self, c):
        """Segment c (from the plan's ground states for c = 0)."""
        psi_in = None if c == 0 else self.psi[(c - 1) % 2]
        psi_out = self.psi[c % 2] if c + 1 < self.nseg else None
        self.L.tdse_propagate_batch(self.plans[self.lens[c]], self.E[c], psi_in, self.acc[c],
                                    self.xe[c], self.nr[c], psi_out, self.st[c])

    def series(self, rows, nseg=None):
        """Accelerations of `rows` over segments [0, nseg), as one series
        (each segment's last sample is the next one's first)."""
        nseg = self.nseg if nseg is None else nseg
        idx = self.torch.as_tensor(rows, device=self.dev)
        parts = [self.acc[c][idx][:, :-1] for c in range(nseg - 1)] + [self.acc[nseg - 1][idx]]
        return self.torch.cat(parts, dim=1).cpu().numpy()

    def statuses_clean(self, nseg=None):
        nseg = self.nseg if nseg is None else nseg
        return all(int((self.st[c] != 0).sum()) == 0 for c in range(nseg))

    def close(self):
        for p in self.plans.values():
            p.close()


def timed_steps(torch, solve, steps, warmup, stream):
    """Warm-up, then `steps` timed bench steps (step j runs segment j mod
    nseg); HIP events on the launch stream around every step.  Returns
    (total ms, per-step ms list, grid-point-steps done)."""
    for j in range(warmup):
        solve.run(j % solve.nseg)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for j in range(steps):
        solve.run(j % solve.nseg)
        ev[j + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[j].elapsed_time(ev[j + 1]) for j in range(steps)]
    work = sum(solve.work[j % solve.nseg] for j in range(steps))
    return ev[0].elapsed_time(ev[steps]), per, work


def kernel_shape(plan, n):
    ki = plan.kernel_info(n)
    lay, info = plan.layout(n), plan.launch_info(n)
    return {"points_per_lane": lay.points_per_lane, "lanes": lay.lanes,
            "scan_levels": lay.scan_levels, "systems_per_workgroup": info.systems_per_workgroup,
            "lds_tables": info.lds_tables, "workgroup_lanes": ki.workgroup_lanes,
            "grid": ki.grid, "workgroups_per_cu": ki.workgroups_per_cu,
            "waves_per_simd": ki.waves_per_simd, "max_waves_per_simd": 8,
            "lds_bytes_per_workgroup": ki.lds_bytes, "vgprs": ki.vgprs}


def lds_bytes_per_point_step(shape):
    """LDS bytes the forward kernel reads per grid-point-step: om is read by
    each of the four sweeps and dV/dx once by the observables (8 B each)
    when both tables are staged in LDS; om alone is staged for the largest
    grids; nothing otherwise."""
    return {1: 40.0, 2: 32.0}.get(shape["lds_tables"], 0.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="volume",
                    choices=["focus", "single", "uneven", "uneven-wide", "volume", "sweep"])
    ap.add_argument("--segments", type=int, default=0,
                    help="time segments of one solve (default: --steps for the volume, so the "
                         "timed steps make up one full solve; 1 otherwise)")
    ap.add_argument("--sweep-n", type=int, default=8192, help="grid size of the sweep workload")
    ap.add_argument("--plain-systems", type=int, default=8)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-focus", action="store_true")
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
    stream = torch.cuda.current_stream()
    opts = 0 if args.no_autotune else L.TDSE_OPT_AUTOTUNE

    w = {"focus": ti.cfg2_focus, "single": ti.cfg1_single, "uneven": ti.cfg3_uneven,
         "uneven-wide": lambda: ti.cfg3_uneven(wide=True),
         "volume": ti.cfg5_volume,
         "sweep": lambda: ti.size_sweep(args.sweep_n)}[args.workload]()
    nseg = args.segments or (args.steps if args.workload == "volume" else 1)
    a_sc, e_g = L.tdse_soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0, tol=1e-13)
    log(f"workload {w.name}: P={w.batch} nt={w.nt} in {nseg} segment(s); soft-core "
        f"a={a_sc:.10f} (E_g={e_g:.13f})")
    t0 = time.time()
    solve = SegmentedSolve(torch, L, w, a_sc, nseg, opts, dev)
    shapes = {n: kernel_shape(solve.plan(), n) for n in sorted(set(w.n_per))}
    log(f"plans built in {time.time() - t0:.2f} s "
        f"({'default layouts' if args.no_autotune else 'autotuned'}), segments of "
        f"{sorted(set(solve.lens))} steps; {len(shapes)} sizes, first {next(iter(shapes.items()))}")

    t_wall = time.perf_counter()
    ms_total, per_ms, work = timed_steps(torch, solve, args.steps, args.warmup, stream)
    t_wall = time.perf_counter() - t_wall
    ms_step = ms_total / args.steps
    value = work / (ms_total * 1e-3)
    clean = solve.statuses_clean(min(args.steps, solve.nseg))
    log(f"batched: {ms_step:.1f} ms/step, {value:.4e} grid-point-steps/s (wall {t_wall:.2f} s "
        f"incl. warm-up); statuses clean: {clean}")
    # the dominant kernel: one forward launch per step (graph replay with a
    # counter reset of a few microseconds)
    avg_launch_s = float(np.mean(per_ms)) * 1e-3
    avg_work = work / args.steps
    achieved = FLOPS_PER_POINT_STEP * avg_work / avg_launch_s / 1e12
    shape0 = next(iter(shapes.values()))
    lds_b = lds_bytes_per_point_step(shape0) if len(shapes) == 1 else None
    lds = None
    if lds_b:
        lds_rate = lds_b * avg_work / avg_launch_s / 1e12
        lds = {"bytes_per_grid_point_step": lds_b, "achieved_tbs": lds_rate,
               "peak_tbs": LDS_PEAK_TBS, "frac": lds_rate / LDS_PEAK_TBS}

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
        "config": {"workload": w.name, "systems": w.batch,
                   "grid_points": int(w.n_per[0]) if len(shapes) == 1 else "ragged",
                   "nt": w.nt, "dx": w.dx, "dt": w.dt,
                   "grid_point_steps": float(sum(w.n_per)) * w.nt,
                   "segments": solve.nseg, "segment_steps": sorted(set(solve.lens)),
                   "timed_grid_point_steps": work,
                   "step": ("one time segment of the solve for every system (psi carried from "
                            "segment to segment); the timed steps make up one full solve"
                            if solve.nseg == args.steps and solve.nseg > 1 else
                            "one full solve of the batch" if solve.nseg == 1 else
                            f"one of {solve.nseg} time segments of the solve"),
                   "parallelism": "single-gpu", "autotune": not args.no_autotune,
                   "layout": shape0 if len(shapes) == 1 else f"{len(shapes)} sizes"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": read_traffic(w.name),
                     "kernel": "forward_kernel (graph replay incl. counter reset)",
                     "flops_per_grid_point_step": FLOPS_PER_POINT_STEP,
                     "grid_point_steps_per_launch": avg_work,
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "lds": lds,
                     "occupancy": {k: shape0[k] for k in ("waves_per_simd", "max_waves_per_simd",
                                                          "workgroups_per_cu", "workgroup_lanes",
                                                          "vgprs", "lds_bytes_per_workgroup")}},
        "statuses_clean": clean,
    }

    # ---------------------------------------------------------- plain form
    if not args.no_plain:
        m = min(args.plain_systems, w.batch)
        rows = list(range(m))
        n0 = solve.lens[0]
        pp_params = L.make_params(w.dx, w.dt, a_sc, n0, mask_fraction=w.mask_frac,
                                  mask_power=w.mask_pow)
        pp = L.Plan(pp_params, [w.n_per[r] for r in rows], options=L.TDSE_OPT_PLAIN)
        Ep = solve.E[0][:m].contiguous()
        ap_ = torch.empty_like(Ep)
        L.tdse_propagate_batch(pp, Ep, None, ap_)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        L.tdse_propagate_batch(pp, Ep, None, ap_)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_plain = e0.elapsed_time(e1)
        ps_plain = float(sum(w.n_per[r] for r in rows)) * n0
        v_plain = ps_plain / (ms_plain * 1e-3)
        same = bool(torch.equal(ap_, solve.acc[0][:m]))
        out["plain"] = {"value": v_plain, "unit": "grid-point-steps/s", "systems_timed": m,
                        "steps": n0, "ms": ms_plain, "batched_over_plain": value / v_plain,
                        "bitwise_equal_to_batched": same}
        log(f"plain: {v_plain:.4e} grid-point-steps/s on {m} systems x {n0} steps; "
            f"batched/plain = {value / v_plain:.1f}")
        pp.close()

    # ------------------------------------------------------------- focus
    focus = None
    if not args.no_focus and args.workload != "focus":
        wf = ti.cfg2_focus()
        a_f = a_sc if wf.dx == w.dx else L.tdse_soft_core_for_ip(wf.ip, 2048, wf.dx, dtau=1.0,
                                                                   tol=1e-13)[0]
        focus = SegmentedSolve(torch, L, wf, a_f, 1, opts, dev)
        ms_f, per_f, work_f = timed_steps(torch, focus, 3, 1, stream)
        v_f = work_f / (ms_f * 1e-3)
        fl_f = FLOPS_PER_POINT_STEP * (work_f / 3) / (np.mean(per_f) * 1e-3) / 1e12
        out["focus"] = {"workload": wf.name, "systems": wf.batch, "nt": wf.nt,
                        "value": v_f, "unit": "grid-point-steps/s", "ms_per_solve": ms_f / 3,
                        "frac": fl_f / FP64_VECTOR_PEAK_TFLOPS,
                        "traffic": read_traffic(wf.name),
                        "layout": kernel_shape(focus.plan(), wf.n_per[0]),
                        "statuses_clean": focus.statuses_clean()}
        log(f"focus: {ms_f / 3:.1f} ms per solve, {v_f:.4e} grid-point-steps/s")

    # ------------------------------------------------------------ adjoint
    if not args.no_adjoint:
        wa = ti.cfg4_adjoint() if args.adjoint_workload == "adjoint" else ti.cfg5_axis()
        a_adj = a_sc if wa.dx == w.dx else L.tdse_soft_core_for_ip(wa.ip, 2048, wa.dx, dtau=1.0,
                                                                     tol=1e-13)[0]
        pa = L.make_params(wa.dx, wa.dt, a_adj, wa.nt, mask_fraction=wa.mask_frac,
                           mask_power=wa.mask_pow)
        plan_a = L.Plan(pa, wa.n_per, adjoint_k=256, options=L.TDSE_OPT_STORE_CHECKPOINTS | opts)
        lay_a = plan_a.layout(wa.n_per[0])
        Ea = wa.efield(xp={"device": dev}).contiguous()
        acc_a = torch.empty_like(Ea)
        h_lo, h_hi = wa.meta["band"]
        k_lo, nk = L.tdse_harmonic_band(wa.nt, wa.dt, wa.omega, h_lo, h_hi)
        work_y = torch.empty(2 * wa.batch * max(nk, 1), dtype=torch.float64, device=dev)
        yld = torch.empty(wa.batch, dtype=torch.float64, device=dev)
        abar = torch.empty_like(Ea)
        grad = torch.empty_like(Ea)

        def gradient(stored):
            # forward (stores the checkpoints), loss gradient, reverse sweep; or
            # the adjoint call that runs its own forward pass again
            L.tdse_propagate_batch(plan_a, Ea, None, acc_a)
            L.tdse_harmonic_yield(wa.batch, wa.nt, wa.dt, wa.omega, h_lo, h_hi, acc_a, None, work_y,
                                  yld, abar)
            if stored:
                L.tdse_adjoint_batch_stored(plan_a, plan_a.checkpoint_generation(), Ea, abar, grad)
            else:
                L.tdse_adjoint_batch(plan_a, Ea, None, abar, grad)

        ms = {}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for stored in (True, False):
            gradient(stored)
            torch.cuda.synchronize()
            e0.record(stream)
            gradient(stored)
            e1.record(stream)
            torch.cuda.synchronize()
            ms[stored] = e0.elapsed_time(e1)
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
                          "forward_grid_point_steps": pts_a,
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
        if not args.no_cpu and args.adjoint_workload == "adjoint":
            out["adjoint"].update(adjoint_cpu_leg(wa, grad.cpu().numpy(), h_lo, h_hi,
                                                  args.cpu_threads))
            log(f"adjoint, cpu oracle: {out['adjoint']['cpu_baseline']['seconds']:.1f} s for "
                f"{out['adjoint']['cpu_baseline']['systems']} systems on "
                f"{out['adjoint']['cpu_baseline']['cores']} threads; gradient parity max rel-L2 "
                f"{out['adjoint']['parity']['grad_rel_l2_max']:.2e}")
        plan_a.close()

    # ------------------------------------------------- energy distribution
    if not args.no_spectrum:
        host = focus if focus is not None else (solve if args.workload == "focus" else None)
        if host is not None:
            out["energy_spectrum"] = bench_spectrum(torch, L, host.plan(), host.w, dev, stream)
            log(f"energy spectrum: {out['energy_spectrum']['ms']:.2f} ms for "
                f"{out['energy_spectrum']['solves']:.0f} (system, energy) solves")
    if focus is not None:
        focus.close()

    # ------------------------------------------------------------ far field
    if not args.no_far_field:
        out["far_field"] = bench_far_field(torch, L, ti, dev, stream)
        log(f"far field: {out['far_field']['ms']:.2f} ms, adjoint {out['far_field']['adjoint_ms']:.2f} ms "
            f"({out['far_field']['terms']:.3g} source-observation-frequency terms)")

    # ------------------------------------------------------- CPU baseline
    if not args.no_cpu:
        import oracle

        cpu = cpu_model()
        # the GPU machine allots 16 host threads to a one-GPU job
        nth = args.cpu_threads or max(1, min(16, cpu["threads_available"]))
        # a stratified sample: the hottest system, the smallest and the
        # largest grid, and rows spread over the batch; one per thread
        by_n = np.argsort(np.asarray(w.n_per), kind="stable")
        picks = {int(np.argmax(w.e0)), int(by_n[0]), int(by_n[-1])}
        n_rows = min(w.batch, max(32, nth))
        picks |= set(np.linspace(0, w.batch - 1, n_rows).round().astype(int).tolist())
        rows = np.array(sorted(picks))[:max(n_rows, 3)]
        # over a bounded number of segments: about ten seconds of CPU time per
        # thread at the oracle's rate of a few 1e7 grid-point-steps/s per core
        n_max = max(w.n_per[r] for r in rows)
        budget = 4.0e8 * nth / (len(rows) * n_max)
        cseg, steps_cpu = 0, 0
        while cseg < solve.nseg and (cseg == 0 or steps_cpu + solve.lens[cseg] <= budget):
            steps_cpu += solve.lens[cseg]
            cseg += 1
        cseg = min(cseg, args.steps)
        steps_cpu = sum(solve.lens[:cseg])
        # the oracle's own soft-core fit and ground states (outside the timing)
        a_ref = oracle.soft_core_for_ip(w.ip, 2048, w.dx, dtau=1.0)[0]
        gs = {}
        psi_list = []
        for r in rows:
            n = w.n_per[r]
            if n not in gs:
                gs[n] = oracle.ground_state(n, w.dx, a_ref, dtau=1.0, tol=1e-14)[0]
            psi_list.append(gs[n])
        e_rows = np.ascontiguousarray(w.efield(rows=rows, nt=steps_cpu))
        t0 = time.perf_counter()
        ref = oracle.propagate_batch(e_rows, psi_list, w.dx, w.dt, a_ref, mask_frac=w.mask_frac,
                                     mask_pow=w.mask_pow, nthreads=nth)
        t_cpu = time.perf_counter() - t0
        ps_cpu = float(sum(w.n_per[r] for r in rows)) * steps_cpu
        # one core: the first sampled system alone over a tenth of the window
        st1 = max(1, steps_cpu // 10)
        t1 = time.perf_counter()
        oracle.propagate_batch(e_rows[:1, :st1 + 1], psi_list[:1], w.dx, w.dt, a_ref,
                               mask_frac=w.mask_frac, mask_pow=w.mask_pow, nthreads=1)
        t1 = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": ps_cpu / t_cpu, "unit": "grid-point-steps/s", "cores": nth,
                               "kind": "oracle",
                               "sample": f"{len(rows)} systems of the same batch (the hottest, the "
                                         f"smallest and largest grid, the rest spread over it), "
                                         f"first {steps_cpu} of {w.nt} steps "
                                         f"({cseg} of {solve.nseg} segments), the systems spread "
                                         f"over {nth} threads, {t_cpu:.1f} s",
                               "single_core_value": float(w.n_per[rows[0]]) * st1 / t1,
                               "cpu": cpu,
                               "full_workload_estimate_s": float(sum(w.n_per)) * w.nt / (ps_cpu / t_cpu),
                               "full_workload_estimate": "extrapolated linearly in grid-point-steps "
                                                         "from the sample's rate"}
        got = solve.series(rows.tolist(), cseg)
        errs = [float(np.linalg.norm(got[i] - ref["accel"][i]) / np.linalg.norm(ref["accel"][i]))
                for i in range(len(rows))]
        out["parity"] = {"accel_rel_l2_max": max(errs), "systems_checked": len(rows),
                         "samples_checked": steps_cpu + 1, "tolerance": 1e-9,
                         "oracle_side": "own soft-core fit and ground state"}
        log(f"cpu oracle: {ps_cpu / t_cpu:.3e} grid-point-steps/s on {nth} threads "
            f"({out['cpu_baseline']['single_core_value']:.3e} on one core, {cpu['model']}); "
            f"parity max rel-L2 {max(errs):.2e} over {len(rows)} systems x {steps_cpu} steps")

    solve.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
