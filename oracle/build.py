"""Build the oracle's C evaluator (test infrastructure) with gcc.

The library is written next to its source as ``libddoracle.so``.  Flags keep
IEEE double semantics: no fused multiply-add contraction, no fast-math.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ddeval.c")
LIB = os.path.join(HERE, "libddoracle.so")
CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-Wall", "-Wextra", "-Wno-unused-function"]


def build(force: bool = True, extra_flags=(), out: str | None = None) -> str:
    out = out or LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force=True, extra_flags=sys.argv[1:]))
