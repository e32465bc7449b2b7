"""CPU-only sanitizer builds: the oracle (gcc) and the host side of the
library (hipcc; the address and undefined-behaviour sanitizers on host code
only) run their small drivers in tests/sanitize/, which exercise every
oracle entry point on small problems and the C ABI's host paths (sizes,
argument validation, refusals before any device work).  A sanitizer report
fails the run (non-zero exit)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1108_1688_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, cwd, timeout):
    res = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)
    return res.returncode, res.stdout + res.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    rc, out = _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-std=c99", "-Wall", "-o", exe,
                    os.path.join(HERE, "oracle_checks.c"), "-lm"], str(tmp_path), 300)
    assert rc == 0, out
    rc, out = _run([exe], str(tmp_path), 300)
    assert rc == 0 and "0 failures" in out and "Sanitizer" not in out, out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="no hipcc")
def test_host_abi_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    srcs = [os.path.join(HERE, "host_checks.cpp")] + [os.path.join(CSRC, f) for f in
                                                      ("hjm_kernels.hip", "hjm_host.hip", "hjm_mlp.hip")]
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", exe, *srcs], str(tmp_path), 900)
    assert rc == 0, out
    rc, out = _run([exe], str(tmp_path), 300)
    assert rc == 0 and "0 failures" in out and "Sanitizer" not in out, out
