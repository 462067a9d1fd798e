"""Build the oracle's shared object (test infrastructure only).

Compiles ``oracle/forces.c`` with gcc into ``oracle/liboracle.so``.  The
flags keep the arithmetic as written (no FMA contraction) and target a
baseline x86-64 level that every current server CPU runs.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "forces.c")
OUT = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-march=x86-64-v3",
          "-ffp-contract=off", "-fno-math-errno", "-std=c11", "-Wall"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
