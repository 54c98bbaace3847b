"""Build libccgmg.so in-tree: the host set-up (C++17) with g++, the HIP
kernels and driver for gfx950 with hipcc, linked into one shared library."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libccgmg.so")
ARCH = os.environ.get("CCGMG_ARCH", "gfx950")


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    host_o = []
    for src in ("setup.cpp", "quadrature.cpp"):
        o = os.path.join(bdir, src.replace(".cpp", ".o"))
        _run(["g++", "-std=c++17", "-O2", "-fPIC", "-pthread", "-Wall", "-I", INCLUDE, "-c",
              os.path.join(CSRC, src), "-o", o])
        host_o.append(o)
    hip_o = os.path.join(bdir, "ccgmg.o")
    _run([hipcc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-c", os.path.join(CSRC, "ccgmg.hip"), "-o", hip_o])
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, hip_o] + host_o + ["-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
