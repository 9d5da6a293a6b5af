"""Compile the oracle's C part (oracle/kapply.c) into oracle/libkqr_oracle.so.

TEST INFRASTRUCTURE: the library serves the FP64 certificates only.

    python -m oracle.build_c

Plain gcc, baseline x86-64 code (no -march=native, so the library runs on any
host the tests run on), no fast-math and no contraction of a * b + c into
fused operations, so every product and sum is one IEEE FP64 rounding.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kapply.c")
LIB = os.path.join(HERE, "libkqr_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", SRC, "-o", tmp,
           "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC}:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
