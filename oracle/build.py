"""Compile the FP64 C oracle into oracle/liboracle.so (test infrastructure only)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fno-semantic-interposition",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp",
           os.path.join(HERE, "oracle.c"), os.path.join(HERE, "oracle_r0.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
