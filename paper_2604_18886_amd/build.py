"""Build the solver's shared library (libmfmg.so) in-tree for gfx950.

    python -m paper_2604_18886_amd.build

Host topology code is compiled with the host compiler and strict IEEE
semantics (no floating-point contraction); the HIP translation unit is
compiled for gfx950 with packed FP32 instructions disabled.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmfmg.so")
ARCH = os.environ.get("MFMG_OFFLOAD_ARCH", "gfx950")


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    topo_o = os.path.join(bdir, "topology.o")
    _run(["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra"] + inc + ["-c", os.path.join(CSRC, "topology.cpp"), "-o", topo_o])
    hip_o = os.path.join(bdir, "mfmg.o")
    _run([hipcc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-Wall", "-Wno-unused-result"] + inc +
         ["-c", os.path.join(CSRC, "mfmg.hip"), "-o", hip_o])
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, topo_o, hip_o])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
