"""Build the HIP library ``libamrvac.so`` in-tree for gfx950.

Every kernel source under ``csrc/`` is compiled with hipcc for gfx950 only,
with packed-FP32 instruction selection disabled (see the design notes), and
linked with the host runtime into one shared library exporting the C ABI of
``include/amrvac.h``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libamrvac.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["fused5.hip", "fused5_hllc.hip", "fused5_hlld.hip", "fused.hip", "plain.hip", "runtime.cpp"]
FLAGS = ["--offload-arch=gfx950", "-Rpass-analysis=kernel-resource-usage", "-ffp-contract=on", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics"]


def build(verbose: bool = False, jobs: int = 6) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC] + FLAGS + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            p, c = procs.pop(0)
            if p.wait() != 0:
                raise subprocess.CalledProcessError(p.returncode, c)
    for p, c in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, c)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
