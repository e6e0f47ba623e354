"""Compile the oracle's C core (md_oracle.c) into _md_oracle.so next to it.

Test infrastructure: the oracle is built alongside the HIP library but is never
linked into it.  Flags: -O2, OpenMP, and -ffp-contract=off so that no
multiply-add is fused (the oracle evaluates each definition operation by
operation).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "md_oracle.c")
OUT = os.path.join(HERE, "_md_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=gnu11", "-Wall", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
