"""Compile the oracle's C sources into shared libraries (gcc, OpenMP):
``wilson_oracle.c`` -> ``oracle/liboracle.so`` and ``staggered_oracle.c`` ->
``oracle/libstaggered_oracle.so``.

Test infrastructure only: building the checker is not using it.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wilson_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
STAG_SRC = os.path.join(HERE, "staggered_oracle.c")
STAG_LIB = os.path.join(HERE, "libstaggered_oracle.so")


def build_oracle(force: bool = False, src: str = SRC, out: str = LIB) -> str:
    stale = (not os.path.exists(out)) or os.path.getmtime(out) < os.path.getmtime(src)
    if force or stale:
        tmp = out + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def build_all(force: bool = False) -> list:
    return [build_oracle(force), build_oracle(force, STAG_SRC, STAG_LIB)]


if __name__ == "__main__":
    print(build_all(force=True))
