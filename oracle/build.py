"""Compile the C oracle into two shared libraries (double and long double).

Test infrastructure only: the GPU library never links these.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gpr_oracle.c")
LIBS = {
    "double": os.path.join(HERE, "liboracle_f64.so"),
    "long double": os.path.join(HERE, "liboracle_ld.so"),
}


def build(verbose: bool = False) -> None:
    """Always recompiles both builds (no -ffast-math: it changes rounding)."""
    for real, out in LIBS.items():
        tmp = out + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
               f"-DOR_REAL={real}", SRC, "-o", tmp, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build(verbose=True)
