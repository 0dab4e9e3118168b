"""Compile the CPU oracle (test infrastructure only) into oracle/libdk_oracle.so.

The Gaussian transform is defined as an exact sequence of binary32 operations, so the
library is built without floating-point contraction and without fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dk_oracle.c")
LIB = os.path.join(HERE, "libdk_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fno-math-errno", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv))
