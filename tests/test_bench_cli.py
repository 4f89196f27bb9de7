"""Host-side checks of the benchmark script: it refuses more than one GPU
with a message, and it reports HBM traffic only for the kernel sources the
committed counter summary was taken from."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    digest = bench.source_digest()
    assert digest == bench.source_digest() and len(digest) == 64
    body = ("copy_bytes = 1073741824\ncopy_fetch_kib = 524288\ncopy_write_kib = 1048576\n"
            "fetch_kib_per_dispatch = 1000\nwrite_kib_per_dispatch = 3000\n")
    (tmp_path / "forward_kernel_w_hbm_traffic.txt").write_text(f"source_sha256 = {digest}\n" + body)
    (tmp_path / "forward_kernel_x_hbm_traffic.txt").write_text("source_sha256 = 0\n" + body)
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    # fetch scaled by 2 (the copy's read counter saw half the bytes), write by 1
    assert bench.read_traffic("w") == 1024.0 * (2 * 1000 + 3000)
    assert bench.read_traffic("x") is None
    assert bench.read_traffic("missing") is None


def test_segments_cover_the_time_loop_once():
    """The headline run splits one solve into time segments: the lengths add
    up to the pulse's steps, differ by at most one, and each segment starts
    where the previous one ended."""
    for nt, k in [(213056, 20), (213056, 64), (44093, 1), (7, 20), (100, 3)]:
        lens = bench.seg_lengths(nt, k)
        assert sum(lens) == nt
        assert max(lens) - min(lens) <= 1
        assert len(lens) == min(k, nt)
