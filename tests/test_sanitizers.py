"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the FP64 oracle (every entry
point on small scenes with degenerate Gaussians, frames, samples and finite differences), and
the host-side argument checks of the HIP library (its host code instrumented, the device code
unchanged; no kernel is launched). Each driver must run clean and exit 0."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_driver")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "oracle", "gs_oracle.cpp"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    assert "oracle driver: ok" in _run(exe)


@pytest.mark.skipif(shutil.which("/opt/rocm/bin/hipcc") is None, reason="needs hipcc")
def test_library_host_checks_under_address_and_undefined_behaviour_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    csrc = os.path.join(ROOT, "paper_2509_17513_amd", "csrc")
    from paper_2509_17513_amd.build import SOURCES
    lib = os.path.join(BUILD, "libgs4d_san.so")
    cmd = ["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", csrc] + [os.path.join(csrc, f) for f in SOURCES] + ["-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = os.path.join(BUILD, "abi_driver")
    # a plain host program (the same clang as the library's host pass, so one sanitizer runtime)
    cmd = ["/opt/rocm/lib/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"), lib,
           "-Wl,-rpath," + BUILD, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "abi driver: ok" in _run(exe)
