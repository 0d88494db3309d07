"""Nearest-neighbour stencils and RBF-FD interpolation weights (Sec. 2.2).

The paper interpolates with cubic polyharmonic splines phi(r) = r^3
(Sec. 2.2, Eq. 13) augmented with the polynomials of total degree two, over
the N_L nearest Eulerian nodes.  The interpolation weights w_j of a point p
are the solution of the symmetric saddle-point system

    [ Phi   P ] [ w  ]   [ phi(|x_j - p|) ]
    [ P^T   0 ] [ mu ] = [ pi(p)          ]

with Phi_jl = |x_j - x_l|^3 and P_jm = pi_m(x_j), pi = (1, x, y, x^2, xy, y^2),
so that sum_j w_j g(x_j) is the value at p of the interpolant of g.
"""
import numpy as np


def min_image(d, box, periodic):
    """Minimum-image displacement: along a periodic axis of length L a component
    larger than L/2 in magnitude is shifted by -sign(d) L."""
    d = np.array(d, dtype=np.float64, copy=True)
    for a in range(2):
        if periodic[a]:
            L = box[a]
            big = d[..., a] > 0.5 * L
            small = d[..., a] < -0.5 * L
            d[..., a] = np.where(big, d[..., a] - L, np.where(small, d[..., a] + L, d[..., a]))
    return d


def nearest(xy, i, K, box, periodic):
    """The K nearest nodes of node i (itself included), by brute force.

    Order: squared distance computed as dx*dx + dy*dy in FP64, ties broken by
    the offset vector (dx, then dy).  The offset tie-break makes the choice
    translation invariant on a regular lattice.  Returns (indices (K,),
    offsets x_j - x_i (K, 2))."""
    d = min_image(xy - xy[i], box, periodic)
    r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    # every node not farther than the K-th smallest distance is a candidate,
    # so ties at the cut are all present before the full ordering
    cut = np.partition(r2, K - 1)[K - 1]
    cand = np.nonzero(r2 <= cut)[0]
    order = cand[np.lexsort((d[cand, 1], d[cand, 0], r2[cand]))]
    sel = order[:K]
    return sel, d[sel]


def nearest_to_point(xy, i, o, K, box, periodic):
    """The K nearest nodes of the point p = x_i + o, ordered like nearest():
    squared distance, then the offset x_j - p (dx, then dy).  The offsets are
    formed as (x_j - x_i) - o, so on a lattice every node's point sees the
    same offsets (and the same ties) whatever the rounding of x_i + o.
    Returns (indices (K,), offsets x_j - p (K, 2))."""
    d = min_image(xy - xy[i], box, periodic) - np.asarray(o, dtype=np.float64)
    r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    cut = np.partition(r2, K - 1)[K - 1]
    cand = np.nonzero(r2 <= cut)[0]
    order = cand[np.lexsort((d[cand, 1], d[cand, 0], r2[cand]))]
    sel = order[:K]
    return sel, d[sel]


def poly2(p):
    """Monomials of total degree <= 2 at points p (..., 2) -> (..., 6)."""
    x, y = p[..., 0], p[..., 1]
    return np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], axis=-1)


def phs3(r):
    """Cubic polyharmonic spline phi(r) = r^3 (Sec. 2.2, Eq. 13)."""
    return r ** 3


def interpolation_weights(X, P, snap=1e-12):
    """Weights w (m, K) with sum_j w[i, j] g(x_j) = s(P_i), s the PHS3 + P2
    interpolant through the stencil nodes X (K, 2), for m evaluation points
    P (m, 2).  X and P are offsets from a common origin; they are divided by
    the stencil radius R first (the weights do not change under this scaling,
    the conditioning does).  If P_i coincides with a node (closer than
    snap * R) the interpolant's value there is that node's value, and the
    unit weight vector is returned exactly."""
    X = np.asarray(X, dtype=np.float64)
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    K = X.shape[0]
    R = np.max(np.hypot(X[:, 0], X[:, 1]))
    if R == 0.0:
        raise ValueError("degenerate stencil")
    Xs = X / R
    Ps = P / R
    diff = Xs[:, None, :] - Xs[None, :, :]
    Phi = phs3(np.hypot(diff[..., 0], diff[..., 1]))
    Pm = poly2(Xs)
    A = np.zeros((K + 6, K + 6))
    A[:K, :K] = Phi
    A[:K, K:] = Pm
    A[K:, :K] = Pm.T
    rp = np.hypot(Xs[None, :, 0] - Ps[:, None, 0], Xs[None, :, 1] - Ps[:, None, 1])  # (m, K)
    B = np.concatenate([phs3(rp), poly2(Ps)], axis=1)                              # (m, K+6)
    w = np.linalg.solve(A, B.T).T[:, :K]
    for i in range(P.shape[0]):
        j = int(np.argmin(rp[i]))
        if rp[i, j] < snap:
            w[i] = 0.0
            w[i, j] = 1.0
    return w
