"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C built with gcc.  -ffp-contract=off keeps every
multiply and add a separate IEEE operation; no -march flag is given, so the
code runs on any x86-64 host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "aqr_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = [
        "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-Wno-unused-parameter", SRC, "-o", tmp, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
