"""The batch schedulers (csrc/coro.h, csrc/sched.hip) under ThreadSanitizer.

Builds csrc/sched.hip and tests/sched_threads.hip for the host only, with
ThreadSanitizer and without the HIP runtime (the test program defines the stream,
event and copy calls on a thread that plays the device), and runs the
program: several host threads meet at one rendezvous in lock-step rounds, in
open rounds and in open rounds whose PCG steps hand their completion through
the tag in the fit's pinned buffer; every K-apply result is checked, and a
launch that fails part-way must stop every thread.  A data race makes
ThreadSanitizer fail the run.
"""
import os
import subprocess
import tempfile

import pytest

from paper_2510_07929_amd import build as kbuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2510_07929_amd", "csrc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not (os.path.exists(CLANGXX) and os.path.exists(kbuild.HIPCC)), reason="no ROCm clang")
def test_schedulers_under_thread_sanitizer():
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in (os.path.join(CSRC, "sched.hip"), os.path.join(HERE, "sched_threads.hip")):
            obj = os.path.join(d, os.path.basename(src) + ".o")
            subprocess.run([kbuild.HIPCC, "-std=c++20", "-O1", "-g", f"--offload-arch={kbuild.ARCH}",
                            "--cuda-host-only", "-Xarch_host", "-fsanitize=thread",
                            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj],
                           check=True, capture_output=True)
            objs.append(obj)
        exe = os.path.join(d, "sched_threads")
        link = [CLANGXX, "-fsanitize=thread", *objs, "-o", exe]
        subprocess.run(link, check=True, capture_output=True)
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
        for seed in ("1", "2", "3"):
            r = subprocess.run([exe, seed], capture_output=True, text=True, env=env, timeout=120)
            report = r.stdout + r.stderr
            assert "ThreadSanitizer" not in report, report[-6000:]
            assert r.returncode == 0 and "schedulers ok" in r.stdout, report[-6000:]
