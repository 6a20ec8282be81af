"""Build the CPU oracle (plain C, two precisions) in place.

Test infrastructure: called by the test suite, the smoke check and the
benchmark's CPU-baseline leg, and by the package build step (building the
checker is not using it).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
         "-shared", "-Wall"]
TARGETS = {"liboracle32.so": [], "liboracle64.so": ["-DORC_DOUBLE"]}


def build(verbose=False):
    src = os.path.join(HERE, "oracle.c")
    for name, extra in TARGETS.items():
        out = os.path.join(HERE, name)
        cmd = ["gcc"] + FLAGS + extra + ["-o", out + ".tmp", src, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def ensure_built():
    src = os.path.join(HERE, "oracle.c")
    for name in TARGETS:
        out = os.path.join(HERE, name)
        if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
            build()
            return


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
