"""Unit conversions and the memory model of the paper (host helpers).

Reynolds-number control by the streaming distance (Sec. 2.3): with fixed
lattice velocity and viscosity, the reference length in lattice units is
L / dx, so Re grows as dx shrinks; keeping the physical viscosity fixed makes
the time step scale as dx^2 (diffusive scaling).
"""
from __future__ import annotations

CS2 = 1.0 / 3.0


def delta_x(h_ref: float, s: float) -> float:
    """Streaming distance for a streaming-distance scale s: dx = h_ref / s, so
    s = h / dx is the factor alpha_E = 1 / alpha_delta of Sec. 2.3 (s = 1 is
    the lattice case dx = h)."""
    return h_ref / s


def nu_lattice(tau_plus: float) -> float:
    """nu_lb = c_s^2 (tau+ - 1/2) (Sec. 2.1, Eq. 6)."""
    return CS2 * (tau_plus - 0.5)


def tau_for_nu(nu_lb: float) -> float:
    return nu_lb / CS2 + 0.5


def reynolds(u_lb: float, length: float, dx: float, tau_plus: float) -> float:
    """Re = U L / nu in lattice units, L counted in streaming distances
    (Sec. 2.3, Eq. 16; Sec. 3.1, Eq. 20)."""
    return u_lb * (length / dx) / nu_lattice(tau_plus)


def tau_for_reynolds(u_lb: float, length: float, dx: float, re: float) -> float:
    return tau_for_nu(u_lb * (length / dx) / re)


def time_step(dx: float, nu_phys: float, tau_plus: float) -> float:
    """dt such that nu_phys = nu_lb dx^2 / dt (Sec. 2.3)."""
    return nu_lattice(tau_plus) * dx * dx / nu_phys


def acceleration_phys(g_lb: float, dx: float, dt: float) -> float:
    """g = g_lb dx / dt^2 (conversion factor C_g, Sec. 2.3)."""
    return g_lb * dx / (dt * dt)


def memory_lbm1(n_nodes: float, n_fields: int = 3) -> float:
    """M_LBM1 / c = 2 N_f N (Sec. 3.2, Eq. 26): two copies of each field."""
    return 2.0 * n_fields * n_nodes


def memory_mlbm1(n_rbf: float, n_lag: float, n_fields: int = 3, q: int = 9,
                 stencil_rbf: int = 25, stencil_lag: int = 9) -> float:
    """M_MLBM1 / c (Sec. 3.2, Eq. 27): the fields plus, for each of the q - 1
    departure points of every node, the weights (one number each) and the
    stencil indices (half a number each, int vs double)."""
    return (2.0 * n_fields * (n_rbf + n_lag)
            + 1.5 * (stencil_rbf * n_rbf + stencil_lag * n_lag) * (q - 1))


def memory_ratio(m_mlbm1: float, m_lbm1: float) -> float:
    """r_M = M_MLBM1 / M_LBM1 (Sec. 3.2, Eq. 28)."""
    return m_mlbm1 / m_lbm1


def lbm1_nodes(porosity: float, dx: float) -> float:
    """Lattice sites of LBM1 in a unit sample: round(phi / dx^2) (Sec. 3.2)."""
    return float(round(porosity / (dx * dx)))


def algorithmic_bytes_per_node(variant: int, storage: int, k_padded: int, weights16: bool = False) -> int:
    """Bytes one node update must move between HBM and the chip in the packed
    device layout: read and write of its own state, its weights, its stencil
    indices and its flags (gathered neighbour state counted once, at the
    owner).  The state is what the method stores: nine populations, or the
    three fields (rho, u, v) of MLBM1 (the device layout pads these to four
    for 16-byte loads; the padding is layout, not algorithm).  variant 0 =
    populations, 1 = fields; storage 0 F64, 1 F32, 2 F16S, 3 BF16;
    weights16: FP16 weights (16-bit states)."""
    tb = {0: 8, 1: 4, 2: 2, 3: 2}[storage]
    wb = 8 if storage == 0 else (2 if weights16 else 4)
    state = (9 if variant == 0 else 3) * tb
    return 2 * state + 8 * k_padded * wb + 4 * k_padded + 2


def block_centre_bytes_per_node(variant: int, storage: int) -> int:
    """The same for a block centre of a hybrid set: its eight neighbour
    indices replace the stencil indices, and its weights are shared by all
    block centres (read once per launch, not per node)."""
    tb = {0: 8, 1: 4, 2: 2, 3: 2}[storage]
    state = (9 if variant == 0 else 3) * tb
    return 2 * state + 8 * 4 + 2


def f16_scale_exp(u_ref: float, target: float = 1024.0) -> int:
    """Power-of-two scale for FP16 offset storage: the stored value is
    offset * 2^sigma, chosen so that an offset of the size of the reference
    velocity u_ref maps to about `target` (well inside FP16's normal range,
    ~60x below its largest value).  Population offsets are at most ~u/3 and
    field offsets ~u, so both stay representable with margin."""
    import math

    return int(math.floor(math.log2(target / abs(u_ref))))
