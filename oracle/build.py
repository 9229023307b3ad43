"""Build the C oracle into ``oracle/_h2_oracle.so`` (test infrastructure only).

The oracle is compiled with ``-ffp-contract=off`` so that its floating-point
results (tree geometry, admissibility decisions) do not depend on whether the
compiler fuses multiply-adds.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "h2_oracle.c")
LIB = os.path.join(HERE, "_h2_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c99", "-Wall", "-Wno-unused-function",
           "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True), file=sys.stderr)
