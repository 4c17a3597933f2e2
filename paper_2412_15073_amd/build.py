"""Build libjumpmd.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libjumpmd.so")
SOURCES = ["md_chain.hip", "md_kernels.hip", "md_capi.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 instructions stay off: hipcc -O3 would otherwise form
         # v_pk_* FP32 operations from scalar float code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # machine-level loop-invariant code motion hoists the constants of the
         # FP64 math routines out of the chain loops into registers (occupancy)
         "-mllvm", "-disable-machine-licm",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-value",
         "-Wno-unused-result"]


# per-source flags: the jump chains' float arithmetic (the FP32-mixed path and
# the float screen of the FP64 path, whose error bound has ample room) uses
# the hardware square root and reciprocal instead of correctly rounded
# division and square root
SOURCE_FLAGS = {"md_chain.hip": ["-fno-hip-fp32-correctly-rounded-divide-sqrt"]}


def build(verbose: bool = False, out: str = OUT, defines=()) -> str:
    """Compile and link the library; defines: extra -D macros (variants)."""
    objs = []
    tag = "" if out == OUT else "_" + str(abs(hash(out)) % 100000)
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + tag + ".o")
        cmd = ([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS + SOURCE_FLAGS.get(src, [])
               + ["-D" + d for d in defines])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
