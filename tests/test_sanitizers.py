"""Host C and C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* oracle.c with tests/sanitize/oracle_check.c: every oracle entry point on ragged random
  inputs, outputs cross-checked, leaks checked.
* The library's host code (argument validation, the workspace-size queries, the tuning
  candidates) built with host-only sanitizers, driven by tests/sanitize/abi_check.c through
  calls that must be answered before any HIP call; the kernels are compiled for gfx950 as
  usual and never launched.  Leak checking is off there: the HIP runtime keeps allocations
  for the life of the process.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _need(tool):
    if not os.path.exists(tool):
        pytest.skip("%s not available" % tool)


def _run(cmd, env=None, cwd=None):
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=cwd)
    return p.returncode, p.stdout + p.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    _need(CLANG)
    exe = str(tmp_path / "oracle_check")
    rc, out = _run([CLANG, "-std=c99"] + SAN + [os.path.join(ROOT, "oracle", "oracle.c"),
                   os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"), "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "runtime error" not in out and "ERROR" not in out, out


def test_abi_validation_under_asan_ubsan(tmp_path):
    _need(CLANG)
    _need(HIPCC)
    csrc = os.path.join(ROOT, "paper_2503_18974_amd", "csrc")
    lib = str(tmp_path / "libmaxsq_san.so")
    host = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer"):
        host += ["-Xarch_host", f]  # sanitizers on the host code only
    rc, out = _run([HIPCC, "-O1", "-fPIC", "-shared", "-std=c++17", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host +
                   [os.path.join(csrc, s) for s in ("kernels.hip", "rect.hip", "cube.hip",
                                                     "api.cpp")] + ["-o", lib])
    assert rc == 0, out
    exe = str(tmp_path / "abi_check")
    rc, out = _run([CLANG, "-std=c99"] + SAN + [os.path.join(ROOT, "tests", "sanitize",
                                                             "abi_check.c"),
                   "-L", str(tmp_path), "-lmaxsq_san", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "runtime error" not in out, out
    assert "all statuses as documented" in out
