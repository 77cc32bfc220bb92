"""Compile the plain-C oracle (liboracle.so) with gcc.  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")

# x86-64-v3 (AVX2/FMA) runs on every host of the target machines; -ffp-contract=off
# keeps each multiply and add separately rounded, exactly as written.
CFLAGS = ["-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build_flags() -> list:
    """The gcc flags the oracle library is built with (reported beside its timing)."""
    return list(CFLAGS)


def build(verbose: bool = False) -> str:
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
