"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU oracle
and of the library's host code, run on the CPU: every oracle entry point on
small inputs (threads included), and the library's argument validation,
status strings and host-side checks (calls refused before any device use,
so no GPU is needed).  A memory error, leak or undefined operation makes
the run fail."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = "/opt/rocm"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(cmd, cwd, env=None, timeout=600):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "oracle_smoke")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, "-o", exe,
          os.path.join(HERE, "oracle_smoke.c"), os.path.join(ROOT, "oracle", "tdse_ref.c"),
          "-lm", "-lpthread"], str(tmp_path))
    r = _run([exe], str(tmp_path))
    assert "oracle smoke: ok" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("the ROCm compilers are not available")
    from paper_2507_04115_amd import build as hip_build

    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    objs = []
    procs = []
    for src in hip_build.SOURCES:
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(
            [hipcc, *hip_build.FLAGS, "-O1", "-g", *host_san, "-c",
             os.path.join(hip_build.CSRC, src), "-o", obj],
            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        out, err = p.communicate(timeout=900)
        assert p.returncode == 0, err
    drv = str(tmp_path / "host_smoke.o")
    _run([clang, "-std=c++17", "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(HERE, "host_smoke.cpp"), "-o", drv], str(tmp_path))
    exe = str(tmp_path / "host_smoke")
    _run([clang, *SAN, "-o", exe, drv, *objs, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
          f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"], str(tmp_path))
    env = dict(os.environ)
    # the HIP runtime keeps allocations for the life of the process
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = _run([exe], str(tmp_path), env=env)
    assert "host smoke: ok" in r.stdout
