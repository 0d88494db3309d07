"""The standard lattice LBM and LBM1 on a periodic n x n lattice (Sec. 2.1).

Used only as fixed points of comparison: with the streaming distance equal to
the lattice spacing, the departure points of the meshless schemes are lattice
nodes and MLBM / MLBM1 must reduce to these.

Populations are (9, n, n) arrays indexed [k, iy, ix]; fields (n, n) and
(n, n, 2).  The flat node id iy * n + ix matches nodesets.regular_grid.
"""
import numpy as np

from . import lattice as lt


def shift(a, k):
    """a evaluated at x - e_k on the periodic lattice: out[x] = a[x - e_k]."""
    return np.roll(a, shift=(int(lt.E[k, 1]), int(lt.E[k, 0])), axis=(0, 1))


def step(f, tau_plus, tau_minus, g=(0.0, 0.0)):
    """Collide (Sec. 2.1, Eq. 3) then stream by index shift (Sec. 2.1, Eq. 1):
    f_k(t+1, x) = f_k^post(t, x - e_k)."""
    n = f.shape[1]
    fpost = lt.collide(f.reshape(9, -1), tau_plus, tau_minus, g).reshape(9, n, n)
    return np.stack([shift(fpost[k], k) for k in range(9)])


def lbm1_step(rho, u, g=(0.0, 0.0)):
    """LBM1 (Sec. 2.1, Eqs. 10-11): the new fields are the zeroth and first
    moments of the equilibria (plus half the force term) of the neighbouring
    nodes' fields, rho(t+1, x) = sum_k f_k^eq(rho(x - e_k), u(x - e_k))."""
    n = rho.shape[0]
    g = np.asarray(g, dtype=np.float64)
    fl = rho.reshape(-1)
    ul = u.reshape(-1, 2)
    src = (lt.equilibrium(fl, ul) + 0.5 * lt.guo_force(fl, ul, g)).reshape(9, n, n)
    fnew = np.stack([shift(src[k], k) for k in range(9)])
    rho_new = fnew.sum(axis=0)
    mom = np.stack([(fnew * lt.E[:, 0, None, None]).sum(0), (fnew * lt.E[:, 1, None, None]).sum(0)], -1)
    u_new = (mom + 0.5 * rho_new[..., None] * g) / rho_new[..., None]
    return rho_new, u_new
