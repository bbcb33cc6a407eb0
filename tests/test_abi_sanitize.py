"""The library's host code under AddressSanitizer and UBSan: the C ABI built
with the sanitizers on its host side only (the device part is compiled but never run),
and a C program that calls every entry point answering before the device is
touched (sizes, status strings, thresholds, every argument error of the
lattice, batch, labeling, server and cubic-lattice calls)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


def test_abi_host_code_clean_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    csrc = os.path.join(ROOT, "paper_1105_5804_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    lib = str(tmp_path / "libswccl_asan.so")
    # the sanitizer applies to the host pass only (every -fsanitize is behind -Xarch_host)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                    "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", inc, "-o", lib, os.path.join(csrc, "swccl.hip"), os.path.join(csrc, "server.hip"),
                    os.path.join(csrc, "cubic.hip")],
                   check=True, capture_output=True, timeout=600)
    exe = str(tmp_path / "abi_exercise")
    subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", inc,
                    os.path.join(ROOT, "tests", "sanitize", "abi_exercise.c"), lib,
                    "-Wl,-rpath," + str(tmp_path), "-lm", "-o", exe],
                   check=True, capture_output=True, timeout=120)
    # leaks of the HIP runtime's own start-up are not this library's
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip() == "ok"
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr
