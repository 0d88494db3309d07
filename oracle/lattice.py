"""D2Q9 lattice quantities and the collision operator (Sec. 2.1).

Populations are arrays of shape (9, n); velocities of shape (n, 2).
"""
import numpy as np

# Streaming vectors e_k in the paper's order (Sec. 2.1, Eq. 2).
E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
              [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.float64)

# Lattice weights omega_k (Sec. 2.1, the equation following Eq. 7).
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)

# Speed of sound squared, c_s = 1/sqrt(3) (Sec. 2.1, after Eq. 6).
CS2 = 1.0 / 3.0


def opposite(k: int) -> int:
    """Index k' of the vector antiparallel to e_k (Sec. 2.1, after Eq. 1),
    found by searching the table rather than hard-coding it."""
    for j in range(9):
        if E[j, 0] == -E[k, 0] and E[j, 1] == -E[k, 1]:
            return j
    raise ValueError(k)


OPP = np.array([opposite(k) for k in range(9)])


def equilibrium(rho, u):
    """f^eq_k(rho, u) of Sec. 2.1, Eq. 7: second-order Hermite equilibrium.

    rho: (n,), u: (n, 2)  ->  (9, n)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    feq = np.empty((9,) + rho.shape)
    usq = u[..., 0] ** 2 + u[..., 1] ** 2
    for k in range(9):
        eu = E[k, 0] * u[..., 0] + E[k, 1] * u[..., 1]
        feq[k] = W[k] * rho * (1.0 + eu / CS2 + eu * eu / (2 * CS2 * CS2) - usq / (2 * CS2))
    return feq


def density(f):
    """rho = sum_k f_k (Sec. 2.1, Eq. 9)."""
    return f.sum(axis=0)


def momentum(f):
    """sum_k f_k e_k (Sec. 2.1, Eq. 9 times rho)  ->  (n, 2)."""
    return np.stack([(f * E[:, 0:1]).sum(axis=0), (f * E[:, 1:2]).sum(axis=0)], axis=-1)


def velocity(f, g):
    """Velocity with a constant body acceleration g: u = (sum_k f_k e_k + rho g / 2) / rho.

    Without forcing this is Eq. 9 of Sec. 2.1.  With forcing, the half-step
    shift belongs to the second-order forcing scheme the paper uses for the
    porous flow (Sec. 3.2); it is read here as Guo's scheme."""
    rho = density(f)
    return (momentum(f) + 0.5 * rho[:, None] * np.asarray(g)[None, :]) / rho[:, None]


def guo_force(rho, u, g):
    """Guo's discrete body-force term, second order in velocity:
    F_k = omega_k [ (e_k - u)/c_s^2 + (e_k . u) e_k / c_s^4 ] . rho g.

    The paper states only that the constant acceleration is discretised to
    second order in the velocities (Sec. 3.2); this is the standard term with
    that property.  Returns (9, n)."""
    g = np.asarray(g, dtype=np.float64)
    F = np.empty((9,) + np.shape(rho))
    for k in range(9):
        eu = E[k, 0] * u[..., 0] + E[k, 1] * u[..., 1]
        cx = (E[k, 0] - u[..., 0]) / CS2 + eu * E[k, 0] / (CS2 * CS2)
        cy = (E[k, 1] - u[..., 1]) / CS2 + eu * E[k, 1] / (CS2 * CS2)
        F[k] = W[k] * rho * (cx * g[0] + cy * g[1])
    return F


def sym_antisym(a):
    """(a_k + a_k')/2 and (a_k - a_k')/2 (Sec. 2.1, Eq. 4)."""
    return 0.5 * (a + a[OPP]), 0.5 * (a - a[OPP])


def collide(f, tau_plus, tau_minus, g=(0.0, 0.0)):
    """TRT collision of Sec. 2.1, Eq. 3 with the split of Eq. 4, plus the body
    force split the same way and weighted by (1 - 1/(2 tau)) per part.

    BGK is the special case tau_minus = tau_plus.  Returns f^post (9, n)."""
    rho = density(f)
    u = velocity(f, g)
    feq = equilibrium(rho, u)
    F = guo_force(rho, u, g)
    fp, fm = sym_antisym(f)
    ep, em = sym_antisym(feq)
    Fp, Fm = sym_antisym(F)
    return (f - (fp - ep) / tau_plus - (fm - em) / tau_minus
            + (1.0 - 0.5 / tau_plus) * Fp + (1.0 - 0.5 / tau_minus) * Fm)


def tau_minus_from_lambda(tau_plus: float, magic: float) -> float:
    """tau^- from Lambda = (tau^+ - 1/2)(tau^- - 1/2) (Sec. 2.1, Eq. 5)."""
    return 0.5 + magic / (tau_plus - 0.5)


def viscosity(tau_plus: float) -> float:
    """nu_lb = c_s^2 (tau^+ - 1/2) (Sec. 2.1, Eq. 6)."""
    return CS2 * (tau_plus - 0.5)
