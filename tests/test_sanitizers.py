"""CPU runs of native host code under sanitizers.

The oracle (plain C) is built with AddressSanitizer and
UndefinedBehaviorSanitizer together with a driver (tests/sanitize_oracle.c)
that exercises every phase, mechanism kind, voltage mode and variant on
random meshes and trees with arrays allocated at their exact sizes.  The
host side of the GPU library is built the same way with a driver
(tests/sanitize_host.cpp) over its host-only entry points; the replay of the
tree cut in test_cable_plan.py checks what that code computes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "tests", "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "mech_oracle.c"),
           "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtimes not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "all finite" in r.stdout


def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    """The host-only entry points of libmech (tree cutting, layouts, the
    node-index check) with the host side of the library built under ASan and
    UBSan; the device code is compiled as usual and never launched."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_1905_02241_amd", "csrc")
    exe = str(tmp_path / "sanitize_host")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-munsafe-fp-atomics",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(ROOT, "tests", "sanitize_host.cpp"), os.path.join(csrc, "mech_kernels.hip"),
           os.path.join(csrc, "mech_runtime.hip"), "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
           "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # leak checking is off: the HIP runtime keeps its own allocations to exit
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    assert ", 0 failed" in r.stdout
