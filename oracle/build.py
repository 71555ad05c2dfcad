"""Compile the plain-C oracle (``ntt_ref.c``) into ``libntt_ref.so``.

Test infrastructure: run by ``__graft_entry__.build()`` and by the tests
when the library is missing. Uses gcc -O2 with OpenMP, no intrinsics.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ntt_ref.c")
LIB = os.path.join(HERE, "libntt_ref.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra",
           SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
