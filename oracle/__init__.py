"""CPU oracle for the meshless lattice Boltzmann method (MLBM / MLBM1).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 numpy
implementation of what the GPU library computes, written from the paper
(Strzelczyk & Matyka, "Modeling inertial flows with meshless Lattice
Boltzmann Method", arXiv 2312.14789) and pinned by the `-m "not gpu"` tests
to closed forms, exact special cases and the paper's printed numbers.  Only
the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it; the library never does, and this package imports nothing from the
library.  Both sides take their inputs from the seeded generators in
`nodesets`.

Modules
  lattice  D2Q9 constants, equilibrium, moments, Guo forcing, TRT collision
           (Sec. 2.1).
  rbf      nearest-neighbour stencils and cubic polyharmonic-spline weights
           with degree-2 polynomial augmentation (Sec. 2.2).
  mlbm     departure points and bounce-back rules, the MLBM step (collide all
           nodes, then stream all nodes) and the MLBM1 step (Sec. 2.2, 3.2),
           macroscopic fields and reductions.
  lbm      the standard lattice LBM and LBM1 on a periodic square lattice
           (Sec. 2.1), used only to pin the meshless step at s = 1.

Parity status: every function is pinned.  The wall force (momentum
exchange, not in the paper) is pinned by the steady momentum balance of a
channel and by the one-step momentum budget of a periodic sample with disks,
where the rest-state subtraction matters; the Dirichlet overwrite by plane
Couette flow (exact on the lattice at tau = 1) and by flows between Dirichlet
lines converging to their closed forms; the permeability formula by the
plane channel's k = H^2 / 12.
"""
