"""Builds libmlbm.so in-tree: host C++ (stencil builder, packing, errors) with
g++, the gfx950 kernels with hipcc, linked into one shared library."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmlbm.so")
PROBE_LIB = os.path.join(HERE, "libmlbm_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# packed FP32 instructions are disabled in all device code
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-I", INCLUDE, "-I", CSRC]
# host code: no contraction, so the FP64 builder rounds like plain arithmetic
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread", "-I", INCLUDE, "-I", CSRC]

HOST_SOURCES = ["stencil_build.cpp", "mlbm_common.cpp"]
HIP_SOURCES = ["mlbm_step.hip", "unet.hip"]
# a bandwidth measurement helper, linked into a library of its own
PROBE_SOURCES = ["bw_probe.hip"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _link(objs, out):
    tmp = out + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-pthread"])
    os.replace(tmp, out)


def build(verbose: bool = True) -> str:
    """Compiles every source, links LIB and PROBE_LIB; returns LIB's path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    _link(objs, LIB)
    probe_objs = []
    for src in PROBE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        probe_objs.append(obj)
    _link(probe_objs, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
