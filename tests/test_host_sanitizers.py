"""The host runtime (argument checks, tail counts, footprints, status strings)
built with AddressSanitizer and UBSan on the host side only, linked with the
in-tree kernel objects, and driven on the CPU by host_sanitizer_driver.c."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1606_04473_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1606_04473_amd", "_build")
KERNEL_OBJS = ["kernels_trial.o", "kernels_parts.o", "kernels_stream.o", "kernels_metrics.o",
               "kernels_adjoint.o", "kernels_portfolio.o"]
# sanitizers on the host pass only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    missing = [o for o in KERNEL_OBJS if not os.path.exists(os.path.join(BUILD, o))]
    if missing:
        pytest.skip(f"kernel objects not built ({missing}); run __graft_entry__.build()")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    api = str(tmp_path / "ara_api.o")
    drv = str(tmp_path / "driver.o")
    exe = str(tmp_path / "driver")
    # the runtime holds no device code, so its host pass alone is compiled
    subprocess.run([hipcc, "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
                    *SAN, *inc, "-c", os.path.join(CSRC, "ara_api.hip"), "-o", api],
                   check=True, capture_output=True)
    subprocess.run([hipcc, "--cuda-host-only", "-O1", "-g", *SAN, "-x", "c", "-std=c99", *inc, "-c",
                    os.path.join(ROOT, "tests", "host_sanitizer_driver.c"), "-o", drv],
                   check=True, capture_output=True)
    subprocess.run([hipcc, *SAN, "--offload-arch=gfx950", "-o", exe, drv, api,
                    *[os.path.join(BUILD, o) for o in KERNEL_OBJS]], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "ok (0 failures)" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
