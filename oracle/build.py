"""Build the oracle's shared objects (test infrastructure only).

Compiles ``oracle/forces.c`` with gcc into ``oracle/liboracle.so`` and
``oracle/snap.c`` into ``oracle/liboracle_snap.so``.  The flags keep the
arithmetic as written (no FMA contraction) and target a baseline x86-64
level that every current server CPU runs.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "forces.c")
OUT = os.path.join(HERE, "liboracle.so")
SRC_SNAP = os.path.join(HERE, "snap.c")
OUT_SNAP = os.path.join(HERE, "liboracle_snap.so")

CFLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-march=x86-64-v3",
          "-ffp-contract=off", "-fno-math-errno", "-std=c11", "-Wall"]


def _gcc(src, out, verbose):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _gcc(SRC_SNAP, OUT_SNAP, verbose)
    return _gcc(SRC, OUT, verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
