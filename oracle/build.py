"""Build the FP64 CPU reference (test infrastructure) with gcc.

    python oracle/build.py        -> oracle/libmgref.so
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmgref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           os.path.join(HERE, "mgref.c"), "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure() -> str:
    """Build only when the library is missing or older than its sources."""
    src = [os.path.join(HERE, f) for f in ("mgref.c", "mgref.h")]
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in src):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
