"""Compile the CPU oracle (test infrastructure) into oracle/libjumpmd_oracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jumpmd_oracle.c")
OUT = os.path.join(HERE, "libjumpmd_oracle.so")


def build(verbose: bool = False, out: str = OUT, plant: int = 0) -> str:
    """Compile the oracle into `out`; plant > 0 builds the mutant with planted
    mistake `plant` (mutation tests only)."""
    # -O2 without fast-math: IEEE semantics, no reassociation; no FMA contraction
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", f"-DORC_PLANT={int(plant)}", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
