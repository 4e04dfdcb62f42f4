"""Sanitizer builds of the CPU code (no GPU needed).

* The FP64 oracle compiled with AddressSanitizer and UndefinedBehaviorSanitizer
  (g++), loaded by the oracle test files in a child process (the sanitizer
  runtimes preloaded): every pin of the oracle runs under the sanitizers.
* The host construction of the compact layout and link words
  (csrc/layout.hpp), compiled for the host with the same sanitizers and checked
  against a brute-force neighbour computation on seeded random boxes
  (tests/sanitize/layout_check.hip: every computed compact index and byte
  offset is bounds-checked)."""

import os
import shutil
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_lattice.py", "test_oracle_cell.py", "test_oracle_gradient.py", "test_oracle_outflow.py",
                "test_oracle_wss.py", "test_oracle_aniso.py", "test_oracle_d3q27.py"]


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("g++ sanitizer runtimes not installed")
    oracle.build(out_dir=str(tmp_path), sanitize=True)
    env = dict(os.environ, ORACLE_LIB_DIR=str(tmp_path), LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    files = [os.path.join(ROOT, "tests", f) for f in ORACLE_TESTS]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + files, cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=1500)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "failed" not in r.stdout


def test_host_layout_under_address_and_ub_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "layout_check")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2402_10809_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "layout_check.hip"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    r = subprocess.run([exe, "400"], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    print(r.stdout[-1500:], r.stderr[-1500:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "400 random boxes" in r.stdout and " 0 failures" in r.stdout


def test_fp64_power_function_on_the_host(tmp_path):
    """The FP64 x^e of csrc/fp64math.hpp (the Carreau-Yasuda law of the FP64
    passes) against the host C library, relative error below 1e-14."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fp64math_check")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-I", os.path.join(ROOT, "paper_2402_10809_amd", "csrc"),
           os.path.join(ROOT, "tests", "sanitize", "fp64math_check.hip"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
