"""Compile the C oracle into oracle/libcfx_oracle.so with gcc.

Test infrastructure only.  -ffp-contract=off keeps every a*b+c as two
rounded operations; -fopenmp only splits independent rows of a step.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcfx_oracle.so")


def build(verbose: bool = False, src: str | None = None, out: str | None = None) -> str:
    """Compile cfx_oracle.c (or another source, for planted-mistake tests)."""
    src = src or os.path.join(HERE, "cfx_oracle.c")
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    cmd.insert(-1, "-I" + HERE)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
