"""Compile the plain-C KPM oracle (test infrastructure) into oracle/libkpm_oracle.so.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
the result.  Plain ``gcc -O2 -fopenmp``; no architecture-specific flags.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kpm_oracle.c")
LIB = os.path.join(HERE, "libkpm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
