"""Host plan builder under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only; the sanitizers instrument the host pass, no GPU code runs)."""
import os
import shutil
import subprocess

import pytest


def test_plan_builder_under_sanitizers(tmp_path):
    """The host plan builder (validation, hierarchy, shifts, tables, the
    Jacobi eigen-solver, tanh faces) built with AddressSanitizer and
    UndefinedBehaviorSanitizer on the host pass and run over valid layouts
    and invalid descriptors (tests/sanitize/plan_host_driver.cpp)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "plan_host_driver")
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(root, "include"), "-I", os.path.join(root, "paper_2106_03583_amd", "csrc"),
           "-x", "hip", os.path.join(root, "paper_2106_03583_amd", "csrc", "plan.cpp"),
           os.path.join(root, "tests", "sanitize", "plan_host_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "OK (0 failures)" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
