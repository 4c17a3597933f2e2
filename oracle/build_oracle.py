"""Compile the CPU oracle (test infrastructure) into oracle/libjumpmd_oracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jumpmd_oracle.c")
OUT = os.path.join(HERE, "libjumpmd_oracle.so")


def build(verbose: bool = False) -> str:
    # -O2 without fast-math: IEEE semantics, no reassociation; no FMA contraction
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
