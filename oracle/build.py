"""Build the FP64 CPU oracle shared libraries (test infrastructure only).

liboracle.so: plain g++ -O2, no fused multiply-add contraction, no
fast-math, OpenMP over independent blocks.  This is the oracle.

liboracle_fma.so: the same source built with multiply-add contraction
(x86 FMA).  It is the oracle with every a*b+c rounded once instead of twice:
not a reference, but a second sample of how far roundoff alone moves a case
(the tests' parity floor).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amrvac_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")
COMMON = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    for out, extra in ((LIB, ["-ffp-contract=off"]), (LIB_FMA, ["-ffp-contract=fast", "-mfma"])):
        cmd = COMMON + extra + ["-o", out + ".tmp", SRC]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
