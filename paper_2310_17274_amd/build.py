"""Build libmg.so (HIP, gfx950) in-tree.

    python -m paper_2310_17274_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmg.so")
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in
           ["mg_api.hip", "mg_kernels.hip", "mg_lbfgs.hip", "mg_eval_wl.hip"] +
           [f"mg_select_p{pl}.hip" for pl in (1, 2, 4, 8, 16)] + ["mg_select_p16h.hip", "mg_select_packed.hip"] +
           [f"mg_eval_wl_s{slots}g{groups}.hip" for slots, groups in
            ((2, 1), (4, 1), (8, 1), (16, 1), (2, 2), (4, 2), (8, 2), (2, 4), (4, 4))] +
           [f"mg_eval_l{lanes}s{slots}.hip" for lanes in (8, 16) for slots in (4, 8, 16)]]
HEADERS = [os.path.join(CSRC, f) for f in ("mg_internal.h", "mg_device.h", "mg_eval.h", "mg_eval_wl.h",
                                           "mg_solver.h")] + \
          [os.path.join(os.path.dirname(HERE), "include", "mg.h")]
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 (v_pk_*_f32) stays off: hipcc may only emit plain FP32
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source to an object (in parallel), then link libmg.so.
    incremental=True skips a source whose object is newer than it and than
    every header."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    hdr_t = max(os.path.getmtime(h) for h in HEADERS + [__file__])
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        objs.append(obj)
        if incremental and os.path.exists(obj) and \
                os.path.getmtime(obj) > max(hdr_t, os.path.getmtime(src)):
            continue
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        log = open(obj + ".log", "w")
        procs.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), obj + ".log"))
        while sum(p.poll() is None for _, p, _ in procs) >= jobs:
            procs[[p.poll() is None for _, p, _ in procs].index(True)][1].wait()
    failed = False
    for src, p, log in procs:
        p.wait()
        if p.returncode != 0:
            sys.stderr.write(open(log).read())
            failed = True
    if failed:
        raise RuntimeError("hipcc failed compiling libmg sources")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libmg.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
