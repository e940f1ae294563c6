"""Compile the oracle's C source into ``oracle/liboracle.so`` (gcc, OpenMP).

Test infrastructure only: building the checker is not using it.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wilson_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build_oracle(force: bool = False, src: str = SRC, out: str = LIB) -> str:
    stale = (not os.path.exists(out)) or os.path.getmtime(out) < os.path.getmtime(src)
    if force or stale:
        tmp = out + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(force=True))
