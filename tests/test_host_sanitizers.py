"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the C oracle, driven by tests/sanitize/oracle_driver.c over small grids and
  its edge cases (poles, l_max 0, m = l_max, partial m-sets, refused inputs);
* the library's host-side ring planning (the fast-path radix lists and LDS
  layouts, the size-class layouts), driven by tests/sanitize/plan_driver.cpp
  over every ring length up to 16384 (hipcc, sanitizers on the host side
  only; no GPU call).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _run(exe, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", *SAN,
                           "-ffp-contract=off", os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "sht_oracle.c"), "-o", exe, "-lm"])
    assert "oracle driver ok" in _run(exe, tmp_path)


def test_ring_planning_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc missing")
    exe = str(tmp_path / "plan_driver")
    flags = []
    for f in SAN:
        flags += ["-Xarch_host", f] if f.startswith("-fsanitize") or f.startswith("-fno-sanitize") else [f]
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", *flags,
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1010_1260_amd", "csrc"),
                           os.path.join(HERE, "sanitize", "plan_driver.cpp"), "-o", exe])
    assert "plan driver ok" in _run(exe, tmp_path)
