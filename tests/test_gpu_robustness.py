"""Failure handling and caches of the library on the GPU:

* the autotuner's on-disk cache: choices written by one plan are read back
  by the next (a planted valid choice is used as written), while garbage,
  a wrong checksum or a layout that does not fit are ignored, the size is
  timed again and the file rewritten with a valid line;
* a cap on the adjoint workspace (TDSE_MAX_WORKSPACE_BYTES) fails plan
  creation with TDSE_E_NOMEM before anything is allocated;
* graph capture switched off (TDSE_FORCE_CAPTURE_FAILURE) leaves the plan
  on direct launches with bitwise the graph replay's results."""
import numpy as np
import pytest

import oracle_side

pytestmark = pytest.mark.gpu
A_AR = 1.1891671


def fnv1a(text: str) -> int:
    h = 1469598103934665603
    for c in text.encode():
        h ^= c
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _line(key_text, C, T, S, tab, rate):
    body = f"{key_text} : {C} {T} {S} {tab} {float(rate).hex()}"
    return f"{body} # {fnv1a(body):016x}\n"


def _forward(lib, torch, plan, efield):
    E = torch.tensor(efield, device="cuda:0")
    acc = torch.empty_like(E)
    st = torch.full((efield.shape[0],), -1, dtype=torch.int32, device="cuda:0")
    lib.tdse_propagate_batch(plan, E, None, acc, None, None, None, st)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    return acc.cpu().numpy()


def test_autotune_disk_cache_round_trip_and_corrupt_fallback(lib, tmp_path):
    import torch

    n, batch, nt, dx, dt = 2048, 6, 120, 0.2, 0.05
    efield = 0.05 * np.random.default_rng(5).standard_normal((batch, nt + 1))
    p = lib.make_params(dx, dt, A_AR, nt)
    path = tmp_path / "tune.txt"
    lib.tdse_set_tune_cache(str(path))
    try:
        plan_a = lib.Plan(p, [n] * batch, options=lib.TDSE_OPT_AUTOTUNE)
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("tdse-tune 1 ")
        key_text = lines[0].split(" : ")[0]
        assert f" {n} {batch} " in key_text
        choice_a = lines[0].split(" : ")[1].split(" # ")[0].split()
        out_a = _forward(lib, torch, plan_a, efield)
        print(f"  probed choice C,T,S,tab = {choice_a[:4]}, layout {plan_a.layout(n)}", flush=True)

        # a planted valid choice (4 points per lane, tables in global memory)
        path.write_text(_line(key_text, 4, 512, 1, 0, 1.25e11))
        lib.tdse_set_tune_cache(str(path))          # also clears the per-process cache
        plan_b = lib.Plan(p, [n] * batch, options=lib.TDSE_OPT_AUTOTUNE)
        assert plan_b.layout(n).points_per_lane == 4
        info = plan_b.launch_info(n)
        assert info.lds_tables == 0 and info.systems_per_workgroup == 1
        assert info.tuned_rate == 1.25e11
        out_b = _forward(lib, torch, plan_b, efield)

        # corrupt entries: garbage, a wrong checksum, a layout that does not fit
        good_other = _line(key_text.replace(f" {n} {batch} ", f" {n + 256} {batch} "), 8, 320, 1, 1, 2e11)
        good_line = _line(key_text, 8, 256, 2, 1, 3e11)
        body, h = good_line.rstrip("\n").split(" # ")
        bad_hash = f"{body} # {int(h, 16) ^ 1:016x}\n"          # one bit of the checksum off
        no_fit = _line(key_text, 4, 2048, 1, 0, 9e11)       # T = 2048 lanes is not a layout
        path.write_text("garbage\n" + "tdse-tune 1 gfx950 truncated\n" + bad_hash + good_other)
        lib.tdse_set_tune_cache(str(path))
        plan_c = lib.Plan(p, [n] * batch, options=lib.TDSE_OPT_AUTOTUNE)
        assert plan_c.launch_info(n).tuned_rate not in (3e11, 9e11)
        path.write_text(no_fit)
        lib.tdse_set_tune_cache(str(path))
        plan_d = lib.Plan(p, [n] * batch, options=lib.TDSE_OPT_AUTOTUNE)
        assert plan_d.launch_info(n).tuned_rate != 9e11
        lay_d = plan_d.layout(n)
        assert lay_d.lanes <= 1024 and lay_d.lanes * lay_d.points_per_lane >= n
        rewritten = path.read_text().splitlines()
        assert len(rewritten) == 1 and rewritten[0].startswith(key_text + " : ")
        out_d = _forward(lib, torch, plan_d, efield)
    finally:
        lib.tdse_set_tune_cache(None)
    for b in (0, batch - 1):
        ref = oracle_side.propagate(efield[b], n, dx, dt, A_AR, mask_frac=0.1)["accel"]
        for out in (out_a, out_b, out_d):
            assert np.linalg.norm(out[b] - ref) / np.linalg.norm(ref) < 1e-9
    for pl in (plan_a, plan_b, plan_c, plan_d):
        pl.close()


def test_workspace_cap_fails_with_nomem(lib, monkeypatch):
    p = lib.make_params(0.2, 0.05, A_AR, 200)
    monkeypatch.setenv("TDSE_MAX_WORKSPACE_BYTES", "100000")
    with pytest.raises(lib.TDSEError) as ei:
        lib.Plan(p, [4096] * 4, adjoint_k=16)
    assert ei.value.status == lib.TDSE_E_NOMEM
    assert "TDSE_MAX_WORKSPACE_BYTES" in str(ei.value)
    with pytest.raises(lib.TDSEError) as ei:
        lib.Plan(p, [4096] * 4, adjoint_k=16, options=lib.TDSE_OPT_STORE_CHECKPOINTS)
    assert ei.value.status == lib.TDSE_E_NOMEM
    monkeypatch.setenv("TDSE_MAX_WORKSPACE_BYTES", "1e12")
    plan = lib.Plan(p, [4096] * 4, adjoint_k=16)   # fits under a large cap
    plan.close()
    monkeypatch.delenv("TDSE_MAX_WORKSPACE_BYTES")
    lib.Plan(p, [4096] * 4, adjoint_k=16).close()


def test_graph_capture_failure_falls_back_to_direct_launches(lib, monkeypatch):
    import torch

    ns = [512, 2048, 2048, 9000]
    nt, dx, dt = 90, 0.2, 0.05
    efield = 0.06 * np.random.default_rng(8).standard_normal((len(ns), nt + 1))
    p = lib.make_params(dx, dt, A_AR, nt)
    plan_g = lib.Plan(p, ns)
    assert plan_g.graph_state() == 0
    out_g = _forward(lib, torch, plan_g, efield)
    assert plan_g.graph_state() == 1
    monkeypatch.setenv("TDSE_FORCE_CAPTURE_FAILURE", "1")
    plan_f = lib.Plan(p, ns)
    out_f = _forward(lib, torch, plan_f, efield)
    assert plan_f.graph_state() == 2
    monkeypatch.delenv("TDSE_FORCE_CAPTURE_FAILURE")
    out_f2 = _forward(lib, torch, plan_f, efield)      # stays on direct launches
    assert plan_f.graph_state() == 2
    assert np.array_equal(out_f, out_g) and np.array_equal(out_f2, out_g)
    plan_g.close()
    plan_f.close()
