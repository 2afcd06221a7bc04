"""AddressSanitizer + UndefinedBehaviorSanitizer builds, run on the CPU:

* the oracle (oracle/oracle.c) built with gcc and the sanitizers, driven
  through every entry point on small dense and CSR problems
  (tests/sanitize/oracle_driver.c), leak detection on;
* the library's host code (hipcc, sanitizers on the host side only, the
  device code unchanged) driven through its host-only paths: validation,
  error texts, every solver's rejection of bad arguments before any device
  work (tests/sanitize/library_driver.hip).  No GPU is needed.

Any report ends the driver with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(exe, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300,
                       cwd=str(tmp_path))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           "-lm", "-o", exe]
    subprocess.run(cmd, check=True, timeout=300)
    out = _run(exe, tmp_path)
    assert "minnorm q1" in out


@pytest.mark.slow
def test_library_host_code_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "library_driver")
    csrc = os.path.join(ROOT, "paper_2304_12168_amd", "csrc")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "kernels.hip"), os.path.join(csrc, "solver.hip"),
           os.path.join(csrc, "batched.hip"), os.path.join(HERE, "library_driver.hip"),
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-o", exe]
    subprocess.run(cmd, check=True, timeout=900, capture_output=True)
    out = _run(exe, tmp_path)
    assert "0 failures" in out
