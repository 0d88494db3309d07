"""The host part of the library (stencil builder, packing, FP16 weight
rounding, tile packing: threaded C++ over raw arrays) built with
AddressSanitizer and UndefinedBehaviorSanitizer, run on seeded node sets of
every kind the builder handles.  The sanitized driver must finish cleanly and
print the same checksums as the same driver built without sanitizers."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import nodesets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2312_14789_amd", "csrc")
SOURCES = [os.path.join(CSRC, "stencil_build.cpp"), os.path.join(CSRC, "mlbm_common.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "builder_driver.cpp")]
COMMON = ["g++", "-std=c++17", "-ffp-contract=off", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("sanitize")
    plain, san = str(d / "driver_plain"), str(d / "driver_asan_ubsan")
    subprocess.run(COMMON + ["-O2", *SOURCES, "-o", plain], check=True)
    subprocess.run(COMMON + ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                             "-fno-sanitize-recover=undefined", *SOURCES, "-o", san], check=True)
    libs = subprocess.run(["ldd", san], capture_output=True, text=True).stdout
    assert "libasan" in libs and "libubsan" in libs, libs
    return d, plain, san


def _write_input(path, ns, K, dx, lattice_h=0.0, per_departure=False, simple_bb=False):
    disks = np.ascontiguousarray(ns.disks, dtype=np.float64).reshape(-1, 3)
    with open(path, "wb") as f:
        f.write(struct.pack("<qq", ns.n, len(disks)))
        f.write(struct.pack("<8i", K, int(per_departure), int(simple_bb), int(ns.periodic[0]), int(ns.periodic[1]),
                            int(ns.walls_y[0]), int(ns.walls_y[1]), 0))
        f.write(struct.pack("<7d", ns.lo[0], ns.lo[1], ns.hi[0], ns.hi[1], dx, lattice_h, ns.fluid_area()))
        f.write(np.ascontiguousarray(ns.xy, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(ns.kind, dtype=np.uint8).tobytes())
        f.write(disks.tobytes())


CASES = {
    "jittered": lambda: (nodesets.jittered_grid(24, seed=7), 12, 1.0 / 24 / 1.5, {}),
    "channel": lambda: (nodesets.channel(8, 13, jitter=0.2, Lx=0.75, H=1.0), 16, 1.0 / 12 / 2.0, {}),
    "porous": lambda: (nodesets.porous(1500, phi=0.75, seed=4, r_range=(0.05, 0.1)), 16, None, {}),
    "karman": lambda: (nodesets.karman(n_target=1500, seed=5), 16, None, {}),
    "hybrid_pixels": lambda: (nodesets.porous(0, phi=0.8, seed=3, h=1.0 / 40, jitter=0.0, r_range=(0.05, 0.1)),
                              16, 1.0 / 40, {"lattice_h": 1.0 / 40}),
    "per_departure": lambda: (nodesets.karman_paper(h_min=1.0 / 80, h_max=1.0 / 10), 25, 0.14 / 42.0,
                              {"per_departure": True, "simple_bb": True}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_sanitized_builder_is_clean_and_identical(drivers, name):
    d, plain, san = drivers
    ns, K, dx, kw = CASES[name]()
    if dx is None:
        dx = ns.h_min if ns.h_min else ns.h
    inp = str(d / f"{name}.bin")
    _write_input(inp, ns, K, dx, **kw)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=3",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    ref = subprocess.run([plain, inp], capture_output=True, text=True, timeout=300)
    got = subprocess.run([san, inp], capture_output=True, text=True, timeout=300, env=env)
    assert ref.returncode == 0, ref.stderr
    assert got.returncode == 0, got.stderr[-4000:]
    assert "runtime error" not in got.stderr and "Sanitizer" not in got.stderr, got.stderr[-4000:]
    assert got.stdout == ref.stdout
    assert got.stdout.startswith("build ")
