"""Shared helpers of the GPU parity tests: run the oracle and the HIP path on
the same seeded inputs and compare their fields."""
import numpy as np

import nodesets
from oracle import lattice as lt
from oracle import mlbm as omlbm


def oracle_bb(st):
    """Bounce-back bit mask of oracle stencils (bit k-1: source k')."""
    flip = st.src != np.arange(1, 9)[None, :]
    return (flip * (1 << np.arange(8))[None, :]).sum(1).astype(np.uint8)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def rel_max(a, b):
    """Largest node-wise error relative to the largest reference value:
    max_i |a_i - b_i| / max_i |b_i| (catches an error confined to a few
    nodes, which a field norm averages away)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def assert_fields_close(u, u_ref, bar, what=""):
    """Both the field norm and the node-wise maximum within bar."""
    e2, em = rel_l2(u, u_ref), rel_max(u, u_ref)
    assert e2 <= bar, f"{what} rel_l2 {e2:.3e} > {bar:.1e}"
    assert em <= bar, f"{what} rel_max {em:.3e} > {bar:.1e}"
    return e2, em


def morton_reordered(ns):
    """The node set renumbered in Morton (Z) order of its coordinates
    (16-bit cells per axis), so that consecutive nodes are close and a tile's
    halo stays small; a plain renumbering, computed here."""
    import copy

    q = ((ns.xy - ns.lo) / (ns.hi - ns.lo) * 65535.0).astype(np.uint64)

    def spread(v):
        v = v & np.uint64(0xFFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v

    order = np.argsort(spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)), kind="stable")
    out = copy.copy(ns)
    out.xy = ns.xy[order]
    out.kind = ns.kind[order]
    out.bc = ns.boundary_values()[order]
    return out


def initial_fields(ns, seed, amp_u, amp_rho):
    """Smooth seeded fields, with the prescribed values on Dirichlet nodes."""
    L = float(np.max(ns.hi - ns.lo))
    rho, u = nodesets.smooth_fields(ns.xy, seed, amp_u=amp_u, amp_rho=amp_rho, L=L)
    d = ns.kind == nodesets.DIRICHLET
    if np.any(d):
        bc = ns.boundary_values()
        rho[d] = bc[d, 0]
        u[d] = bc[d, 1:3]
    return rho, u


def lagrange_last(ns, st):
    """The node set and the oracle's stencils renumbered so that the block
    centres come after every other node (the order the library's block-centre
    kernel needs); returns (ns, st) in the new order."""
    import copy

    p = np.argsort(st.lagrange, kind="stable")
    inv = np.empty_like(p)
    inv[p] = np.arange(len(p))
    ns2 = copy.copy(ns)
    ns2.xy = ns.xy[p]
    ns2.kind = ns.kind[p]
    if ns.bc is not None:
        ns2.bc = ns.bc[p]
    st2 = omlbm.Stencils(idx=inv[st.idx[p]], w=st.w[p], src=st.src[p], point=st.point[p],
                         area=st.area[p], lagrange=st.lagrange[p])
    return ns2, st2


def run_oracle(ns, st, variant, steps, rho0, u0, tau_plus, tau_minus, g):
    """Oracle fields after `steps` steps: (rho, u)."""
    if variant == 0:
        f = omlbm.init_populations(rho0, u0)
        for _ in range(steps):
            f = omlbm.step(f, ns, st, tau_plus, tau_minus, g)
        return omlbm.macroscopic(f, ns, g), f
    r, u = rho0.copy(), u0.copy()
    for _ in range(steps):
        r, u = omlbm.mlbm1_step(r, u, ns, st, g)
    return (r, u), None


def sim_from_oracle(M, ns, st, variant, storage, tau_plus, tau_minus, g, **kw):
    """Simulation fed with the oracle's own stencil arrays (oracle node order)."""
    # per-departure rows of block centres carry their block weights themselves
    lag = st.lagrange if st.lagrange is not None and st.lagrange.any() and st.idx.ndim == 2 else None
    wl = st.w[int(np.argmax(st.lagrange))][:, :9] if lag is not None else None
    return M.Simulation(st.idx.astype(np.int32), st.w, oracle_bb(st), ns.kind, st.area,
                        variant=variant, storage=storage, tau_plus=tau_plus, tau_minus=tau_minus,
                        g=g, bc=ns.boundary_values(), lagrange=lag, w_lagrange=wl, **kw)


def oracle_one_step_at(ns, nodes, K, dx, variant, rho0, u0, tau_plus, tau_minus, g, lattice_h=None,
                       per_departure=False, simple_bb=False):
    """Fields after one step at the listed nodes only, computed node by node
    with the oracle's own stencil of each node (for node sets too large for a
    whole oracle run).  rho0, u0: initial fields of all nodes."""
    out_r, out_u = [], []
    d_all = ns.kind == nodesets.DIRICHLET
    bc = ns.boundary_values()
    for i in nodes:
        idx, w, src, _, _ = omlbm.stencil_at(ns, i, K, dx, lattice_h, per_departure, simple_bb)
        if idx.ndim == 1:
            idx = np.tile(idx, (8, 1))
        if d_all[i]:
            out_r.append(bc[i, 0])
            out_u.append(bc[i, 1:3])
            continue
        if variant == 0:
            f = np.empty(9)
            for k in range(0, 9):
                cols = np.concatenate([[i], idx[max(k, 1) - 1]])
                f0 = omlbm.init_populations(rho0[cols], u0[cols])
                fpost = lt.collide(f0, tau_plus, tau_minus, g)
                dd = d_all[cols]
                if np.any(dd):
                    fpost[:, dd] = lt.equilibrium(bc[cols[dd], 0], bc[cols[dd], 1:3])
                f[k] = fpost[0, 0] if k == 0 else np.sum(w[k - 1] * fpost[src[k - 1], 1:])
            r = f.sum()
            u = (lt.E.T @ f + 0.5 * r * np.asarray(g)) / r
        else:
            g_ = np.asarray(g)
            own = lt.equilibrium(rho0[[i]], u0[[i]]) + 0.5 * lt.guo_force(rho0[[i]], u0[[i]], g_)
            f = np.empty(9)
            f[0] = own[0, 0]
            for k in range(1, 9):
                mk = idx[k - 1]
                rh = np.sum(w[k - 1] * rho0[mk])
                uh = np.array([[np.sum(w[k - 1] * u0[mk, 0]), np.sum(w[k - 1] * u0[mk, 1])]])
                at = lt.equilibrium(np.array([rh]), uh) + 0.5 * lt.guo_force(np.array([rh]), uh, g_)
                f[k] = at[src[k - 1], 0]
            r = f.sum()
            u = (lt.E.T @ f + 0.5 * r * g_) / r
        out_r.append(r)
        out_u.append(u)
    return np.array(out_r), np.array(out_u)
