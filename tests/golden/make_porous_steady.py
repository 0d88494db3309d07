"""Writes tests/golden/porous_steady_mlbm1.npz: the oracle's steady MLBM1 flow
through a seeded porous sample, the reference of the reduced-storage
steady-state tests.

Calls only the oracle (and the seeded node-set generator): the stored fields
are the FP64 oracle's, never the library's.  The run takes minutes on one
host core, which is why its result is stored instead of being recomputed by
every test run.

Workload: the periodic unit box with random non-overlapping disks (radii
0.04 - 0.07, porosity 0.7, seed 6) and ~1.26e4 nodes, MLBM1 (tau = 1,
Sec. 2.2, Eqs. 14-15), K = 16 shared stencils, streaming distance dx = h
(s = 1), body acceleration g = (2e-6, 0) (Darcy regime), from rest until the
field residual ||u^n - u^(n-100)|| / ||u^n|| falls below 1e-9.

Usage: python tests/golden/make_porous_steady.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import nodesets  # noqa: E402
from oracle import mlbm  # noqa: E402

OUT = os.path.join(HERE, "porous_steady_mlbm1.npz")
PARAMS = dict(n_target=12000, phi=0.7, seed=6, r_range=(0.04, 0.07), K=16, g=2e-6, tol=1e-9, every=100)


def node_set():
    p = PARAMS
    return nodesets.porous(p["n_target"], phi=p["phi"], seed=p["seed"], r_range=p["r_range"])


def xy_digest(xy):
    return hashlib.sha256(np.ascontiguousarray(xy, dtype=np.float64).tobytes()).hexdigest()


def main():
    p = PARAMS
    ns = node_set()
    dx = ns.h
    t0 = time.time()
    st = mlbm.build_stencils(ns, p["K"], dx)
    print(f"{ns.n} nodes, {len(ns.disks)} disks, stencils in {time.time() - t0:.1f} s", flush=True)
    g = (p["g"], 0.0)
    rho, u = np.ones(ns.n), np.zeros((ns.n, 2))
    u_old = u.copy()
    steps, res = 0, np.inf
    while res >= p["tol"]:
        for _ in range(p["every"]):
            rho, u = mlbm.mlbm1_step(rho, u, ns, st, g)
        steps += p["every"]
        red = mlbm.reductions(rho, u, st.area, u_prev=u_old)
        res = red["residual"]
        u_old = u.copy()
        if steps % 1000 == 0:
            print(f"{steps} steps, residual {res:.3e}, {time.time() - t0:.0f} s", flush=True)
    red = mlbm.reductions(rho, u, st.area)
    k = mlbm.permeability(red, 1.0, 1.0 / 6.0, p["g"], dx)
    np.savez_compressed(OUT, rho=rho, u=u, steps=np.int64(steps), residual=np.float64(res),
                        permeability=np.float64(k), n=np.int64(ns.n), xy_sha256=np.array(xy_digest(ns.xy)),
                        g=np.float64(p["g"]), K=np.int64(p["K"]), dx=np.float64(dx))
    print(f"wrote {OUT}: {steps} steps, residual {res:.3e}, permeability {k:.6e}", flush=True)


if __name__ == "__main__":
    main()
