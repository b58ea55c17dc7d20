"""CPU builds of the oracle and of the library's host code with
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

The oracle driver (tests/sanitize/oracle_driver.cpp) runs every
configuration the oracle supports on tiny ragged grids; the host driver
(tests/sanitize/host_driver.cpp) exercises the C ABI's host side
(configuration checks, workspace layout, error texts) of a library whose
host code is instrumented (the device code is unaffected)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(SAN, "oracle_driver.cpp"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout


@pytest.mark.skipif(not shutil.which("/opt/rocm/bin/hipcc") or
                    not os.path.exists("/opt/rocm/lib/llvm/bin/clang++"),
                    reason="ROCm compilers not found")
def test_host_library_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2511_20337_amd", "csrc")
    lib = str(tmp_path / "libmhd_san.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g",
                           "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san +
                          ["-I", os.path.join(ROOT, "include")] +
                          [os.path.join(csrc, f) for f in
                           ("mhd_api.hip", "mhd_kernels.hip", "mhd_adjoint.hip")] + ["-o", lib],
                          stderr=subprocess.DEVNULL)
    # the driver is plain C++: the same clang (and sanitizer runtime), no HIP
    exe = str(tmp_path / "host_driver")
    subprocess.check_call(["/opt/rocm/lib/llvm/bin/clang++", "-std=c++17", "-O1", "-g",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(SAN, "host_driver.cpp"), lib, "-o", exe,
                           "-Wl,-rpath," + str(tmp_path)])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host driver ok" in r.stdout
