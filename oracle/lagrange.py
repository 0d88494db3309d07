"""Biquadratic Lagrange interpolation on the regular part of a hybrid node set
(Sec. 2.2).

The paper discretises the bulk of the fluid on a square lattice and keeps
scattered nodes only where the geometry needs them.  A departure point whose
target node has, as its nine nearest Eulerian nodes, a square 3 x 3 block of
spacing h centred on it, is interpolated with the tensor product of the
quadratic Lagrange polynomials through that block; every other departure
point uses RBF-FD (oracle.rbf).

Member order of a block: member j is the node at x_i + h e_j, with e_j the
D2Q9 velocity j (j = 0 is the node itself).  In units of h the departure
point of population k is t = -(dx / h) e_k, and the weight of member j is
l_{e_j,x}(t_x) l_{e_j,y}(t_y) with the quadratic Lagrange basis through the
abscissae -1, 0, 1:
    l_{-1}(t) = t (t - 1) / 2,   l_0(t) = (1 - t)(1 + t),   l_{+1}(t) = t (t + 1) / 2.
"""
import numpy as np

from . import lattice as lt
from .rbf import nearest


def quadratic_basis(t):
    """Quadratic Lagrange basis through -1, 0, 1 at t: (..., 3) for the
    abscissae -1, 0, +1."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([0.5 * t * (t - 1.0), (1.0 - t) * (1.0 + t), 0.5 * t * (t + 1.0)], axis=-1)


def biquadratic_weights(P, h):
    """Weights (m, 9) of the points P (m, 2), given as offsets from the block
    centre, over the block members in D2Q9 order."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64)) / h
    bx = quadratic_basis(P[:, 0])  # (m, 3)
    by = quadratic_basis(P[:, 1])
    ex = lt.E[:, 0].astype(np.int64) + 1  # column of the basis for each member
    ey = lt.E[:, 1].astype(np.int64) + 1
    return bx[:, ex] * by[:, ey]


def lattice_block(ns, i, h, tol=1e-9):
    """Indices (9,) of the block members of node i in D2Q9 order if its nine
    nearest nodes are exactly x_i + h e_j (each within tol * h) and every other
    node lies farther than the block corners; None otherwise."""
    if ns.n < 9:
        return None
    m = min(10, ns.n)
    sel, off = nearest(ns.xy, i, m, ns.hi - ns.lo, ns.periodic)
    if m == 10:
        d10 = np.hypot(off[9, 0], off[9, 1])
        if d10 <= np.sqrt(2.0) * h * (1.0 + tol):
            return None
    out = np.full(9, -1, dtype=np.int64)
    for j in range(9):
        want = h * lt.E[j]
        err = np.hypot(off[:9, 0] - want[0], off[:9, 1] - want[1])
        a = int(np.argmin(err))
        if err[a] > tol * h:
            return None
        out[j] = sel[a]
    if len(set(out.tolist())) != 9:
        return None
    return out
