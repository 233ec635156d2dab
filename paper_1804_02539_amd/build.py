"""Build libigamg.so in-tree for gfx950 (hipcc for the HIP sources, g++ for the
host setup), and the C oracle helpers if any.  Always recompiles."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libigamg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-march=x86-64-v2",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall",
              "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]


def run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build():
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in ["kernels.hip", "assemble.hip", "coarse.hip", "igamg.hip"]:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    obj = os.path.join(BUILD, "host_setup.o")
    cmd = ["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, "host_setup.cpp"), "-o", obj]
    print(" ".join(cmd), flush=True)
    procs.append(subprocess.Popen(cmd))
    objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise SystemExit("compilation failed")
    tmp = LIB + ".tmp"
    run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs +
        ["-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
