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
HIP_SOURCES = ["mlbm_step.hip", "mlbm_lanes.hip", "unet.hip"]
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
    """Compiles every source (in parallel), links LIB and PROBE_LIB; returns
    LIB's path."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HOST_SOURCES:
        jobs.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")])
    for src in HIP_SOURCES + PROBE_SOURCES:
        jobs.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")])
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(_run, jobs))
    _link([os.path.join(BUILD, s + ".o") for s in HOST_SOURCES + HIP_SOURCES], LIB)
    _link([os.path.join(BUILD, s + ".o") for s in PROBE_SOURCES], PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
