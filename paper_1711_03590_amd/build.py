"""Builds libdg.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled on each call; the per-degree kernel unit inst.hip is
compiled once per number of 1D points (2..9) in parallel.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Wno-unused-function", "-Wno-unknown-pragmas",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]

SOURCES = ["dg_ops.hip", "dg_solver.hip", "dg_batch.hip"]
POINTS = range(2, 10)


def _jobs():
    jobs = []
    for s in SOURCES:
        jobs.append((os.path.join(CSRC, s), os.path.join(BUILD, s.replace(".hip", ".o")), []))
    for n in POINTS:
        jobs.append((os.path.join(CSRC, "inst.hip"), os.path.join(BUILD, f"inst_n{n}.o"), [f"-DDG_N={n}"]))
    return jobs


def _compile(job):
    src, obj, extra = job
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(obj)}:\n{err}")
    return obj, err


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    js = _jobs()
    workers = jobs or min(len(js), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_compile, js))
    if verbose:
        for obj, err in results:
            if err.strip():
                print(f"[{os.path.basename(obj)}]\n{err}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose="-v" in sys.argv))
