"""Builds liboracle.so from oracle.c with gcc (plain C99 + OpenMP, no -ffast-math)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_sanitized() -> str:
    """liboracle_san.so: the same source under AddressSanitizer and
    UndefinedBehaviorSanitizer (gcc, CPU only), for running the pins with
    every out-of-bounds access or undefined operation reported.  Loading it
    into Python needs libasan first in the process (LD_PRELOAD)."""
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle_san.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
