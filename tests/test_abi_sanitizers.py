"""Host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds libkqr with both sanitizers on its host code (the GPU code is built as
always) into a temporary directory, builds tests/abi_sanitize.c with both,
(with the same clang, whose sanitizer runtime the library expects) and runs
it: argument validation, option defaults, status strings, the
tuning-file reader, the test hook and, without a GPU, the no-device status.
A memory or UB error makes the sanitizers abort the driver.
"""
import os
import subprocess
import tempfile

import pytest

from paper_2510_07929_amd import build as kbuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


CLANG = os.path.join(os.path.dirname(os.path.realpath(kbuild.HIPCC)), "..", "llvm", "bin", "clang")
if not os.path.exists(CLANG):
    CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="the ROCm clang is not available")
def test_c_abi_host_code_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "libkqr.so")
        kbuild.build(lib=lib, build_dir=os.path.join(d, "obj"), host_flags=SAN)
        exe = os.path.join(d, "abi_sanitize")
        subprocess.run([CLANG, "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"),
                        os.path.join(HERE, "abi_sanitize.c"), "-o", exe, "-L", d, "-lkqr",
                        f"-Wl,-rpath,{d}"], check=True)
        env = dict(os.environ)
        # the HIP runtime keeps process-lifetime allocations: leaks are not checked
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
        r = subprocess.run([exe, d], capture_output=True, text=True, env=env, timeout=300)
        report = r.stdout + r.stderr
        assert "AddressSanitizer" not in report and "runtime error:" not in report, report[-4000:]
        assert r.returncode == 0, report[-4000:]
        assert "all statuses as expected" in r.stdout
