"""Python binding of libmlbm.so with the names of the C ABI (include/mlbm.h).

Only argument marshalling lives here: numpy arrays for the host builder,
PyTorch tensors for device memory and streams.  Every step of the method runs
in the library (host C++ builder, HIP kernels).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (BF16, F16S, F32, F64, FIELDS, POPULATIONS, RED_COUNT, Batch, DeviceState, Geometry,
                   MlbmError, Sizes, Steady, StencilParams, Stencils, StepParams, check, lib)

__all__ = ["build_stencils", "packed_sizes", "pack_stencils", "Simulation", "MlbmError",
           "POPULATIONS", "FIELDS", "F64", "F32", "F16S", "BF16"]


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def geometry_struct(xy, kind, lo, hi, periodic, walls_y=(False, False), disks=None, fluid_area=0.0):
    """Builds the mlbm_geometry struct; returns (struct, keep-alive arrays)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    disks = np.ascontiguousarray(np.zeros((0, 3)) if disks is None else disks, dtype=np.float64)
    g = Geometry()
    g.n = xy.shape[0]
    g.xy = _ptr(xy)
    g.kind = _ptr(kind)
    g.lo[0], g.lo[1] = float(lo[0]), float(lo[1])
    g.hi[0], g.hi[1] = float(hi[0]), float(hi[1])
    g.periodic[0], g.periodic[1] = int(bool(periodic[0])), int(bool(periodic[1]))
    g.wall_lo_y, g.wall_hi_y = int(bool(walls_y[0])), int(bool(walls_y[1]))
    g.n_disks = disks.shape[0]
    g.disks = _ptr(disks) if disks.shape[0] else None
    g.fluid_area = float(fluid_area)
    return g, (xy, kind, disks)


def build_stencils(xy, kind, lo, hi, periodic, K, dx, walls_y=(False, False), disks=None,
                   fluid_area=0.0, reorder=1, n_threads=0, lattice_h=0.0, per_departure=False,
                   simple_bounce_back=False) -> dict:
    """mlbm_build_stencils: returns perm (n,), idx (n, K) (per_departure:
    (n, 8, K)), w (n, 8, K), bb (n,), area (n,), lagrange (n,) uint8,
    w_lagrange (8, 9) and n_lagrange (lattice_h > 0: hybrid set, block
    centres use the shared weights)."""
    g, keep = geometry_struct(xy, kind, lo, hi, periodic, walls_y, disks, fluid_area)
    n = g.n
    out = {"perm": np.zeros(n, np.int64), "idx": np.zeros((n, 8, K) if per_departure else (n, K), np.int32),
           "w": np.zeros((n, 8, K), np.float64), "bb": np.zeros(n, np.uint8),
           "area": np.zeros(n, np.float64), "lagrange": np.zeros(n, np.uint8),
           "w_lagrange": np.zeros((8, 9), np.float64)}
    st = Stencils(_ptr(out["perm"]), _ptr(out["idx"]), _ptr(out["w"]), _ptr(out["bb"]), _ptr(out["area"]),
                  _ptr(out["lagrange"]), _ptr(out["w_lagrange"]), 0)
    p = StencilParams(K=K, reorder=reorder, dx=float(dx), n_threads=n_threads, lattice_h=float(lattice_h),
                      per_departure=int(bool(per_departure)), simple_bounce_back=int(bool(simple_bounce_back)))
    check(lib.mlbm_build_stencils(ctypes.byref(g), ctypes.byref(p), ctypes.byref(st)))
    out["n_lagrange"] = int(st.n_lagrange)
    del keep
    return out


def build_stencils_for(ns, K, dx, reorder=1, n_threads=0, lattice_h=0.0, per_departure=False,
                       simple_bounce_back=False) -> dict:
    """build_stencils for an object carrying xy, kind, lo, hi, periodic,
    walls_y, disks and fluid_area()."""
    return build_stencils(ns.xy, ns.kind, ns.lo, ns.hi, ns.periodic, K, dx, walls_y=ns.walls_y,
                          disks=ns.disks, fluid_area=ns.fluid_area(), reorder=reorder,
                          n_threads=n_threads, lattice_h=lattice_h, per_departure=per_departure,
                          simple_bounce_back=simple_bounce_back)


def mark_lagrange(lagrange, flags):
    """mlbm_mark_lagrange on host packed flags (in place)."""
    lagrange = np.ascontiguousarray(lagrange, dtype=np.uint8)
    check(lib.mlbm_mark_lagrange(lagrange.shape[0], _ptr(lagrange), _ptr(flags)))
    return flags


def packed_sizes(n, K, variant, storage) -> Sizes:
    s = Sizes()
    check(lib.mlbm_packed_sizes(n, K, variant, storage, ctypes.byref(s)))
    return s


def pack_stencils(idx, w, bb, kind, storage):
    """mlbm_pack_stencils: host arrays in the device layout (idx, w, flags)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    bb = np.ascontiguousarray(bb, dtype=np.uint8)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    n, K = idx.shape
    s = packed_sizes(n, K, POPULATIONS, storage)
    ip = np.zeros(s.idx_bytes, np.uint8)
    wp = np.zeros(s.w_bytes, np.uint8)
    fl = np.zeros(n, np.uint16)
    check(lib.mlbm_pack_stencils(n, K, storage, _ptr(idx), _ptr(w), _ptr(bb), _ptr(kind), _ptr(ip),
                                 _ptr(wp), _ptr(fl)))
    return ip, wp, fl


def weights_to_f16(w_packed, n, k_padded):
    """mlbm_weights_to_f16: FP16 copy (uint16 array) of packed FP32 weights
    (uint8 or float32 host array, layout [8][k_padded/4][n][4]), each row's
    sum kept as closely as FP16 allows."""
    w32 = np.ascontiguousarray(w_packed).view(np.float32)
    if w32.size != 8 * k_padded * n:
        raise ValueError("packed weights do not match n and k_padded")
    out = np.zeros(w32.size, np.uint16)
    check(lib.mlbm_weights_to_f16(n, k_padded, _ptr(w32), _ptr(out)))
    return out


def pack_tiles(idx, tile):
    """mlbm_tile_sizes + mlbm_pack_tiles: (halo_off, halo, lidx, max_halo).
    idx (n, K), or (n, 8, K) for per-departure stencils (each departure
    point's members padded to a multiple of 8 with the node itself)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim == 3:
        n, _, K = idx.shape
        k8 = (K + 7) // 8 * 8
        pad = np.repeat(np.arange(n, dtype=np.int32)[:, None, None], 8, axis=1)
        idx = np.concatenate([idx, np.repeat(pad, k8 - K, axis=2)], axis=2).reshape(n, 8 * k8)
    n, K = idx.shape
    total = ctypes.c_int64()
    mx = ctypes.c_int32()
    check(lib.mlbm_tile_sizes(n, K, tile, _ptr(idx), ctypes.byref(total), ctypes.byref(mx)))
    nt = (n + tile - 1) // tile
    halo_off = np.zeros(nt + 1, np.int32)
    halo = np.zeros(max(total.value, 1), np.int32)
    k8 = (K + 7) // 8 * 8
    lidx = np.zeros(k8 * n, np.uint16)
    check(lib.mlbm_pack_tiles(n, K, tile, _ptr(idx), _ptr(halo_off), _ptr(halo), _ptr(lidx)))
    return halo_off, halo, lidx, mx.value


class Simulation:
    """Device buffers (PyTorch) and parameters of one node set.

    idx, w, bb, area are the builder's arrays in its node order; kind and bc
    (n, 3) must be given in that same order."""

    def __init__(self, idx, w, bb, kind, area, *, variant=POPULATIONS, storage=F32, tau_plus=0.8,
                 tau_minus=None, g=(0.0, 0.0), bc=None, scale_exp=0, block=256, xcd_remap=1,
                 fp32_arith=0, alternate_sweeps=1, cached_weights=0, tile=256, device="cuda",
                 packed=None, lagrange=None, w_lagrange=None, stochastic_rounding=0, weights16=0,
                 hybrid_launches=0, box_area=0.0, graph_steps=0, lanes_per_node=1):
        import torch

        self.torch = torch
        idx = np.asarray(idx)
        self.per_departure = idx.ndim == 3
        n, K = idx.shape[0], idx.shape[-1]
        self.n, self.K = n, K
        if packed is not None:
            ip, wp, fl = packed
        elif self.per_departure:
            # the eight stencils' packed indices one after another, weights as usual
            parts = [pack_stencils(idx[:, k, :], w, bb, kind, storage) for k in range(8)]
            ip = np.concatenate([p_[0] for p_ in parts])
            wp, fl = parts[0][1], parts[0][2]
        else:
            ip, wp, fl = pack_stencils(idx, w, bb, kind, storage)
        self.sizes = packed_sizes(n, K, variant, storage)
        dev = torch.device(device)
        self.wl_d = None
        self.lagrange_begin = n
        if lagrange is not None and w_lagrange is not None and np.any(lagrange):
            lag = np.asarray(lagrange).astype(bool)
            fl = mark_lagrange(lag, fl.copy())
            # the block-centre kernel takes the trailing run of block centres
            self.lagrange_begin = n - int(np.argmin(lag[::-1])) if not lag.all() else 0
            wt = np.float64 if storage == F64 else np.float32
            self.wl_d = torch.from_numpy(np.ascontiguousarray(w_lagrange, dtype=wt)).to(dev)
        self.idx_d = torch.from_numpy(ip).to(dev)
        if weights16:
            if storage not in (F16S, BF16):
                raise MlbmError(-5, "FP16 weights go with 16-bit states only")
            wp = weights_to_f16(wp, n, packed_sizes(n, K, variant, storage).k_padded).view(np.uint8)
        self.w_d = torch.from_numpy(wp).to(dev)
        self.flags_d = torch.from_numpy(fl.view(np.int16)).to(dev)
        if bc is None:
            bc = np.zeros((n, 3))
            bc[:, 0] = 1.0
        self.bc_d = torch.from_numpy(np.ascontiguousarray(bc, dtype=np.float64)).to(dev)
        self.area_d = torch.from_numpy(np.ascontiguousarray(area, dtype=np.float64)).to(dev)
        self.state_d = [torch.zeros(self.sizes.state_bytes, dtype=torch.uint8, device=dev) for _ in range(2)]
        ws = lib.mlbm_reduction_workspace_bytes(n)
        self.ws_d = torch.zeros(max(ws, 8), dtype=torch.uint8, device=dev)
        self.red_d = torch.full((RED_COUNT,), float("nan"), dtype=torch.float64, device=dev)
        self.box_area = float(box_area)
        self.params = StepParams()
        self.params.variant = variant
        self.params.storage = storage
        self.params.tau_plus = float(tau_plus)
        self.params.tau_minus = float(tau_plus if tau_minus is None else tau_minus)
        self.params.g[0], self.params.g[1] = float(g[0]), float(g[1])
        self.params.scale_exp = int(scale_exp)
        self.params.block = int(block)
        self.params.xcd_remap = int(xcd_remap)
        self.params.fp32_arith = int(fp32_arith)
        self.params.alternate_sweeps = int(alternate_sweeps)
        self.params.cached_weights = int(cached_weights)
        self.params.stochastic_rounding = int(stochastic_rounding)
        self.params.weights16 = int(bool(weights16))
        self.params.hybrid_launches = int(hybrid_launches)
        self.params.graph_steps = int(graph_steps)
        self.params.lanes_per_node = int(lanes_per_node)
        self.ds = DeviceState()
        self.ds.n = n
        self.ds.K = K
        self.ds.idx = self.idx_d.data_ptr()
        self.ds.w = self.w_d.data_ptr()
        self.ds.flags = self.flags_d.data_ptr()
        self.ds.bc = self.bc_d.data_ptr()
        self.ds.state[0] = self.state_d[0].data_ptr()
        self.ds.state[1] = self.state_d[1].data_ptr()
        self.ds.cur = 0
        self.ds.w_lagrange = self.wl_d.data_ptr() if self.wl_d is not None else None
        self.ds.lagrange_begin = self.lagrange_begin
        self.ds.per_departure = int(self.per_departure)
        self.set_tile(tile, idx)

    def set_tile(self, tile, idx=None):
        """Selects global gathers (tile 0) or LDS-staged tiles of 64/128/256
        nodes (packs the tile halos from the [n][K] stencil indices)."""
        self.ds.tile = int(tile)
        if tile:
            if idx is None:
                idx = self._idx_host
            halo_off, halo, lidx, mx = pack_tiles(idx, tile)
            t = self.torch
            dev = self.state_d[0].device
            self.halo_off_d = t.from_numpy(halo_off).to(dev)
            self.halo_d = t.from_numpy(halo).to(dev)
            self.lidx_d = t.from_numpy(lidx.view(np.int16)).to(dev)
            self.ds.max_halo = mx
            self.ds.halo_off = self.halo_off_d.data_ptr()
            self.ds.halo = self.halo_d.data_ptr()
            self.ds.lidx = self.lidx_d.data_ptr()
        self._idx_host = np.ascontiguousarray(idx if idx is not None else self._idx_host, dtype=np.int32)

    def _stream(self, stream=None):
        s = stream if stream is not None else self.torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def init_state(self, rho, u, stream=None):
        """mlbm_init_state from host or device FP64 fields rho (n,), u (n, 2)."""
        t = self.torch
        r = t.as_tensor(np.ascontiguousarray(rho, dtype=np.float64) if isinstance(rho, np.ndarray) else rho,
                        dtype=t.float64, device=self.state_d[0].device).contiguous()
        v = t.as_tensor(np.ascontiguousarray(u, dtype=np.float64) if isinstance(u, np.ndarray) else u,
                        dtype=t.float64, device=self.state_d[0].device).contiguous()
        self._keep = (r, v)
        check(lib.mlbm_init_state(ctypes.byref(self.params), ctypes.byref(self.ds), r.data_ptr(),
                                  v.data_ptr(), self._stream(stream)))

    def step(self, nsteps=1, stream=None):
        """mlbm_step."""
        check(lib.mlbm_step(ctypes.byref(self.params), ctypes.byref(self.ds), int(nsteps), self._stream(stream)))

    def macroscopic(self, dx, u_prev=None, want_fields=True, stream=None):
        """mlbm_macroscopic: returns (rho, u, reductions) as device tensors
        (the reductions buffer is reused: its previous mean velocity feeds
        RED_MEAN_CHANGE)."""
        t = self.torch
        dev = self.state_d[0].device
        rho = t.empty(self.n, dtype=t.float64, device=dev) if want_fields else None
        u = t.empty((self.n, 2), dtype=t.float64, device=dev) if want_fields else None
        check(lib.mlbm_macroscopic(ctypes.byref(self.params), ctypes.byref(self.ds), self.area_d.data_ptr(),
                                   float(dx), self.box_area, rho.data_ptr() if rho is not None else None,
                                   u.data_ptr() if u is not None else None,
                                   u_prev.data_ptr() if u_prev is not None else None,
                                   self.ws_d.data_ptr(), self.red_d.data_ptr(), self._stream(stream)))
        return rho, u, self.red_d

    def state_bytes(self):
        """Current state buffer as a host numpy uint8 array (synchronises)."""
        return self.state_d[self.ds.cur].cpu().numpy()

    def run_to_steady(self, dx, tol=1e-6, check_every=100, max_steps=1_000_000, stream=None, criterion="field",
                      hold=1):
        """mlbm_run_to_steady: steps until the residual stays below tol for
        `hold` checks check_every steps apart.  criterion "field":
        ||u^n - u^(n - check_every)|| / ||u^n|| over the nodes; "mean": the
        relative change of the mean velocity (the integral of u_x), the
        paper's steady criterion (Sec. 3.2), which stays meaningful when 16-bit
        storage keeps rounding noise in every node.  Raises MlbmError (code
        MLBM_ERR_UNSTABLE) when a check finds non-finite fields.
        Returns (steps, residual, reductions as numpy)."""
        if criterion not in ("field", "mean"):
            raise ValueError(f"unknown criterion {criterion!r}")
        t = self.torch
        u_prev = t.zeros((self.n, 2), dtype=t.float64, device=self.state_d[0].device)
        sp = Steady(criterion=_lib.STEADY_FIELD if criterion == "field" else _lib.STEADY_MEAN,
                    check_every=int(check_every), hold=int(hold), max_steps=int(max_steps), tol=float(tol))
        red = np.full(RED_COUNT, np.nan)
        done = ctypes.c_int64()
        check(lib.mlbm_run_to_steady(ctypes.byref(self.params), ctypes.byref(self.ds), ctypes.byref(sp),
                                     self.area_d.data_ptr(), float(dx), self.box_area, u_prev.data_ptr(),
                                     self.ws_d.data_ptr(), self.red_d.data_ptr(), _ptr(red), ctypes.byref(done),
                                     self._stream(stream)))
        res = red[_lib.RED_RESIDUAL if criterion == "field" else _lib.RED_MEAN_CHANGE]
        return int(done.value), float(res), red

    # -- checkpoint / resume --------------------------------------------------------

    def save_checkpoint(self, path):
        """Writes the current state buffer, which buffer is current and the
        step count (the key of stochastic rounding) to an .npz file: a run
        resumed from it with load_checkpoint continues bitwise as the
        uninterrupted run would (synchronises)."""
        np.savez(path, state=self.state_bytes(), cur=np.int32(self.ds.cur),
                 step_count=np.uint64(self.ds.step_count), n=np.int64(self.n),
                 variant=np.int32(self.params.variant), storage=np.int32(self.params.storage))

    def load_checkpoint(self, path):
        """Restores a state written by save_checkpoint into this simulation,
        which must have been built for the same node set, variant and storage
        (only plain arrays are read: no pickles)."""
        with np.load(path, allow_pickle=False) as z:
            if (int(z["n"]), int(z["variant"]), int(z["storage"])) != (self.n, self.params.variant,
                                                                       self.params.storage):
                raise ValueError("checkpoint is for another node count, variant or storage")
            state = z["state"]
            if state.size != self.sizes.state_bytes:
                raise ValueError("checkpoint state has the wrong size")
            cur = int(z["cur"])
            self.state_d[cur].copy_(self.torch.from_numpy(np.ascontiguousarray(state)))
            self.ds.cur = cur
            self.ds.step_count = int(z["step_count"])


class BatchSimulation:
    """Many node sets in one concatenated launch (mlbm_batch_init,
    mlbm_step_batched).  Each sample is padded to a multiple of `tile` nodes
    with Dirichlet nodes at rest that have no stencil and zero area, so no tile
    spans two samples.

    samples: list of (stencils dict from build_stencils, kind, bc) with kind
    and bc in the builder's node order."""

    def __init__(self, samples, *, variant=FIELDS, storage=F32, tau_plus=1.0, tau_minus=None,
                 g=(0.0, 0.0), tile=256, check_every=100, grid=0, scale_exp=0, xcd_remap=1,
                 fp32_arith=0, group_bytes=160e6, alternate_sweeps=1, device="cuda"):
        import torch

        self.torch = torch
        if any(np.asarray(st["idx"]).ndim != 2 for st, _, _ in samples):
            raise ValueError("batched runs take one stencil per node (no per-departure stencils)")
        K = samples[0][0]["idx"].shape[1]
        sizes = [st["idx"].shape[0] for st, _, _ in samples]
        pad = self.PAD  # a multiple of every tile size, so any tile stays in one sample
        padded = [(m + pad - 1) // pad * pad for m in sizes]
        off = np.concatenate([[0], np.cumsum(padded)]).astype(np.int64)
        N = int(off[-1])
        self.sizes, self.node_off, self.K, self.N = sizes, off, K, N
        ps = packed_sizes(N, K, variant, storage)
        ip = np.zeros(ps.idx_bytes, np.uint8)
        wp = np.zeros(ps.w_bytes, np.uint8)
        fl = np.zeros(N, np.uint16)
        idx_all = np.empty((N, K), np.int32)
        area_all = np.zeros(N)
        bc_all = np.zeros((N, 3))
        bc_all[:, 0] = 1.0
        for s_, (st, kind, bc) in enumerate(samples):
            a, m, p = int(off[s_]), sizes[s_], padded[s_]
            idx = np.ascontiguousarray(st["idx"], dtype=np.int32) + a
            pad_idx = np.repeat(np.arange(a + m, a + p, dtype=np.int32)[:, None], K, axis=1)
            idx_s = np.concatenate([idx, pad_idx])
            w_s = np.concatenate([st["w"], np.zeros((p - m, 8, K))])
            bb_s = np.concatenate([st["bb"], np.zeros(p - m, np.uint8)])
            kind_s = np.concatenate([np.asarray(kind, np.uint8), np.full(p - m, 2, np.uint8)])
            check(lib.mlbm_pack_stencils_range(N, a, p, K, storage, _ptr(idx_s), _ptr(np.ascontiguousarray(w_s)),
                                               _ptr(bb_s), _ptr(kind_s), _ptr(ip), _ptr(wp), _ptr(fl)))
            idx_all[a:a + p] = idx_s
            area_all[a:a + m] = st["area"]
            if bc is not None:
                bc_all[a:a + m] = bc
        self.sim = Simulation(idx_all, None, None, None, area_all, variant=variant, storage=storage,
                              tau_plus=tau_plus, tau_minus=tau_minus, g=g, bc=bc_all, scale_exp=scale_exp,
                              xcd_remap=xcd_remap, fp32_arith=fp32_arith, tile=tile, device=device,
                              packed=(ip, wp, fl))
        t = torch
        dev = self.sim.state_d[0].device
        ntiles = N // 64  # workspaces sized for the smallest tile
        ns = len(samples)
        self.u_prev_d = t.zeros((N, 2), dtype=t.float64, device=dev)
        self.tile_red_d = t.zeros((ntiles, 4), dtype=t.float64, device=dev)
        self.queue_d = t.zeros(ntiles, dtype=t.int32, device=dev)
        self.counters_d = t.zeros(4, dtype=t.int32, device=dev)
        self.steps_d = t.zeros(ns, dtype=t.int32, device=dev)
        self.res_d = t.zeros(ns, dtype=t.float64, device=dev)
        self.ux_d = t.zeros(ns, dtype=t.float64, device=dev)
        self.batch = Batch()
        b = self.batch
        b.n_samples = ns
        b.check_every = int(check_every)
        b.grid = int(grid)
        b.area = self.sim.area_d.data_ptr()
        b.u_prev = self.u_prev_d.data_ptr()
        b.tile_red = self.tile_red_d.data_ptr()
        b.queue = self.queue_d.data_ptr()
        b.counters = self.counters_d.data_ptr()
        b.sample_steps = self.steps_d.data_ptr()
        b.sample_residual = self.res_d.data_ptr()
        b.sample_int_ux = self.ux_d.data_ptr()
        self.sim.params.alternate_sweeps = int(alternate_sweeps)
        self.set_groups(group_bytes)
        self.stream = torch.cuda.Stream(device=dev)
        self.set_tile(tile)

    def set_groups(self, group_bytes):
        """Consecutive samples grouped so each group's stepping data (state,
        weights, indices) stays under group_bytes (0 = one group)."""
        per_node = packed_sizes(1 << 10, self.K, self.sim.params.variant, self.sim.params.storage)
        bpn = (per_node.w_bytes + per_node.idx_bytes + 2 * per_node.state_bytes) / (1 << 10)
        off = [0]
        acc = 0.0
        for s_, m in enumerate(self.sizes):
            if group_bytes and acc > 0 and acc + m * bpn > group_bytes:
                off.append(s_)
                acc = 0.0
            acc += m * bpn
        off.append(len(self.sizes))
        self.group_bytes = float(group_bytes)
        self.group_off_host = np.asarray(off, np.int32)
        dev = self.sim.state_d[0].device
        self.group_off_d = self.torch.from_numpy(self.group_off_host).to(dev)
        self.group_q_d = self.torch.zeros(len(off), dtype=self.torch.int32, device=dev)
        self.batch.n_groups = len(off) - 1
        self.batch.group_sample_off = self.group_off_d.data_ptr()
        self.batch.group_sample_off_host = self.group_off_host.ctypes.data
        self.batch.group_queue_off = self.group_q_d.data_ptr()

    PAD = 256

    def set_tile(self, tile):
        """Tile size of the LDS-staged persistent kernels (64, 128 or 256)."""
        if tile not in (64, 128, 256):
            raise ValueError("tile must be 64, 128 or 256")
        if self.sim.ds.tile != tile:
            self.sim.set_tile(tile)
        self.tile = tile
        self.tile_off_host = (self.node_off // tile).astype(np.int32)
        self.tile_off_d = self.torch.from_numpy(self.tile_off_host).to(self.sim.state_d[0].device)
        self.batch.sample_tile_off = self.tile_off_d.data_ptr()
        self.batch.sample_tile_off_host = self.tile_off_host.ctypes.data

    def init_state(self, rho_list, u_list):
        """Initial fields per sample (builder order); padding nodes at rest."""
        N = self.N
        rho = np.ones(N)
        u = np.zeros((N, 2))
        for s_, (r, v) in enumerate(zip(rho_list, u_list)):
            a, m = int(self.node_off[s_]), self.sizes[s_]
            rho[a:a + m] = r
            u[a:a + m] = v
        with self.torch.cuda.stream(self.stream):
            self.sim.init_state(rho, u, stream=self.stream)
            check(lib.mlbm_batch_init(ctypes.byref(self.sim.params), ctypes.byref(self.sim.ds),
                                      ctypes.byref(self.batch), ctypes.c_void_p(self.stream.cuda_stream)))

    def run(self, max_steps, tol=1e-6, use_graph=True):
        """mlbm_step_batched; returns the steps run."""
        done = ctypes.c_int32()
        check(lib.mlbm_step_batched(ctypes.byref(self.sim.params), ctypes.byref(self.sim.ds),
                                    ctypes.byref(self.batch), int(max_steps), float(tol), int(bool(use_graph)),
                                    ctypes.byref(done), ctypes.c_void_p(self.stream.cuda_stream)))
        return done.value

    def results(self):
        """(steps to convergence, last residual, sum A u_x) per sample."""
        self.stream.synchronize()
        return self.steps_d.cpu().numpy(), self.res_d.cpu().numpy(), self.ux_d.cpu().numpy()

    def state_of(self, s_):
        """Raw state bytes of sample s_ (its node rows of every state block)."""
        self.stream.synchronize()
        raw = self.sim.state_d[self.sim.ds.cur].cpu().numpy()
        return raw, int(self.node_off[s_]), self.sizes[s_]
