"""Builds the oracle's C part (``bsmm.c`` -> ``libbsmm.so``) with gcc and
OpenMP.  Test infrastructure only: the block-sparse oracle loads the library
when it is present.  Shares nothing with the HIP library's build."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bsmm.c")
LIB = os.path.join(HERE, "libbsmm.so")


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed on {SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
