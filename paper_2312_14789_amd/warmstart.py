"""Learned warm start for porous-media runs.

A network maps the rasterised geometry of a periodic porous sample to the
steady velocity and density field; the MLBM1 run then starts from that field
instead of from rest, and converges to the same steady state (the plain run
from rest is the fallback and the reference its result is checked against).  Training data are steady states the
library itself computes (batched runs); the network is trained on the GPU by
the library's own forward and backward kernels.

Samples: random non-overlapping disks in the unit periodic box on a res^2
pixel grid; the fluid nodes are the centres of the fluid pixels (plus nodes on
every disk surface), so node values and pixel values coincide.
"""
from __future__ import annotations

import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import nodesets

from . import mlbm as M
from . import unet as U


def _make_sample(args):
    seed, res, phi, r_range = args
    ns = nodesets.porous(0, phi=phi, seed=seed, h=1.0 / res, jitter=0.0, r_range=r_range)
    mask = nodesets.raster_mask(ns.disks, res)
    return ns, mask


def make_geometries(n, res=256, seed=231214789, phi_range=(0.6, 0.8), r_range=(0.01, 0.03), workers=8, log=None):
    """n periodic random-disk samples (porosity drawn uniformly from phi_range,
    radii uniform in r_range)."""
    rng = np.random.default_rng(seed)
    jobs = [(int(seed + 1000 + i), res, float(rng.uniform(*phi_range)), tuple(r_range)) for i in range(n)]
    out = []
    ex = ProcessPoolExecutor(max_workers=workers) if workers > 1 else None
    try:
        it = ex.map(_make_sample, jobs, chunksize=4) if ex else map(_make_sample, jobs)
        for i, r in enumerate(it):
            out.append(r)
            if log and (i + 1) % 128 == 0:
                log(f"{i + 1}/{n} geometries")
    finally:
        if ex:
            ex.shutdown()
    return out


def pixel_of_nodes(ns, res):
    """Pixel (row, col) of every fluid grid node, -1 for surface nodes."""
    ix = np.floor(ns.xy[:, 0] * res).astype(np.int64)
    iy = np.floor(ns.xy[:, 1] * res).astype(np.int64)
    grid = ns.kind == nodesets.FLUID
    return np.where(grid, iy, -1), np.where(grid, ix, -1)


def steady_states(samples, g, K=16, tol=1e-6, batch_size=64, max_steps=200_000, check_every=100, log=None):
    """Steady MLBM1 (FP32) fields of every sample, computed in batched runs.
    Returns per sample (rho, u) in the node set's order, and the steps each
    sample needed."""
    out, steps_all = [], []
    for a in range(0, len(samples), batch_size):
        chunk = samples[a:a + batch_size]
        built = [M.build_stencils_for(ns, K, ns.h) for ns, _ in chunk]
        batch = M.BatchSimulation([(b, ns.kind[b["perm"]], None) for b, (ns, _) in zip(built, chunk)],
                                  variant=M.FIELDS, storage=M.F32, tau_plus=1.0, g=(g, 0.0), tile=256,
                                  check_every=check_every)
        batch.init_state([np.ones(b["idx"].shape[0]) for b in built], [np.zeros((b["idx"].shape[0], 2)) for b in built])
        batch.run(max_steps, tol=tol, use_graph=True)
        steps, _, _ = batch.results()
        rho, u, _ = batch.sim.macroscopic(1.0)
        rho = rho.cpu().numpy()
        u = u.cpu().numpy()
        for s_, (b, (ns, _)) in enumerate(zip(built, chunk)):
            o, m = int(batch.node_off[s_]), batch.sizes[s_]
            inv = np.empty(m, np.int64)
            inv[b["perm"]] = np.arange(m)
            out.append((rho[o:o + m][inv], u[o:o + m][inv]))
        steps_all.extend(steps.tolist())
        del batch
        if log:
            log(f"{len(out)}/{len(samples)} steady states")
    return out, steps_all


def converged_only(geoms, fields, steps):
    """The samples whose steady state was reached (steps > 0; 0 = step cap,
    negative = unstable), with the number dropped."""
    keep = [i for i, k in enumerate(steps) if k > 0]
    return [geoms[i] for i in keep], [fields[i] for i in keep], [steps[i] for i in keep], len(steps) - len(keep)


def rasterise(ns, res, rho, u):
    """(target (res, res, 3) = (u_x, u_y, rho - 1), mask (res, res)) from node fields."""
    r, c = pixel_of_nodes(ns, res)
    sel = r >= 0
    t = np.zeros((res, res, 3), np.float32)
    m = np.zeros((res, res), np.float32)
    t[r[sel], c[sel], 0] = u[sel, 0]
    t[r[sel], c[sel], 1] = u[sel, 1]
    t[r[sel], c[sel], 2] = rho[sel] - 1.0
    m[r[sel], c[sel]] = 1.0
    return t, m


class Dataset:
    """Inputs (fluid indicator rasters), normalised targets and loss masks on
    the GPU."""

    def __init__(self, geoms, fields, res, device="cuda"):
        import torch

        n = len(geoms)
        fluid = np.stack([1.0 - g[1] for g in geoms]).astype(np.float32)
        tg = np.zeros((n, res, res, 3), np.float32)
        mk = np.zeros((n, res, res), np.float32)
        for i, ((ns, _), (rho, u)) in enumerate(zip(geoms, fields)):
            tg[i], mk[i] = rasterise(ns, res, rho, u)
        sel = mk > 0
        self.u_scale = float(np.sqrt(np.mean(tg[..., 0][sel] ** 2 + tg[..., 1][sel] ** 2)))
        self.r_scale = float(np.sqrt(np.mean(tg[..., 2][sel] ** 2))) or 1.0
        tg[..., :2] /= self.u_scale
        tg[..., 2] /= self.r_scale
        self.fluid = torch.from_numpy(fluid).to(device)
        self.target = torch.from_numpy(tg).to(device)
        self.mask = torch.from_numpy(mk).to(device)
        self.n, self.res = n, res

    def inputs(self, idx, pad=U.PAD):
        """bf16 bits (len(idx), res, res, pad) with the fluid indicator in channel 0."""
        import torch

        x = torch.zeros((len(idx), self.res, self.res, pad), dtype=torch.bfloat16, device=self.fluid.device)
        x[..., 0] = self.fluid[idx].to(torch.bfloat16)
        return x.view(torch.int16)


def train(net, data, epochs, lr=1e-3, seed=0, log=None):
    """Adam on the masked MSE of the normalised fields; returns the mean loss of
    every epoch."""
    import torch

    rng = np.random.default_rng(seed)
    B = net.batch
    history = []
    for ep in range(epochs):
        order = rng.permutation(data.n)
        tot, cnt = 0.0, 0
        lr_e = lr * (0.5 * (1 + np.cos(np.pi * ep / max(epochs, 1))) * 0.9 + 0.1)
        for a in range(0, data.n - B + 1, B):
            idx = torch.from_numpy(order[a:a + B]).to(data.fluid.device)
            net.forward(data.inputs(idx))
            loss = net.loss_and_grad(data.target[idx].contiguous(), data.mask[idx].contiguous())
            net.backward()
            net.adam_step(lr_e)
            tot += float(loss.item())
            cnt += 1
        history.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep} loss {history[-1]:.5f} lr {lr_e:.2e}")
    return history


def predict(net, data_like, masks_solid, u_scale, r_scale):
    """Network fields (u_x, u_y, rho - 1) for solid masks (list of (res, res)),
    in physical (lattice) units."""
    import torch

    res = masks_solid[0].shape[0]
    out = []
    B = net.batch
    for a in range(0, len(masks_solid), B):
        chunk = masks_solid[a:a + B]
        x = torch.zeros((B, res, res, U.PAD), dtype=torch.bfloat16, device=net.dev)
        for j, m in enumerate(chunk):
            x[j, ..., 0] = torch.from_numpy(1.0 - m).to(net.dev).to(torch.bfloat16)
        y = net.forward(x.view(torch.int16))[..., :3].cpu().numpy()
        for j in range(len(chunk)):
            f = y[j].copy()
            f[..., :2] *= u_scale
            f[..., 2] *= r_scale
            out.append(f)
    return out


def node_fields(ns, res, field):
    """Initial (rho, u) at the nodes from a predicted raster (surface nodes at
    rest with unit density)."""
    r, c = pixel_of_nodes(ns, res)
    sel = r >= 0
    rho = np.ones(ns.n)
    u = np.zeros((ns.n, 2))
    rho[sel] = 1.0 + field[r[sel], c[sel], 2]
    u[sel, 0] = field[r[sel], c[sel], 0]
    u[sel, 1] = field[r[sel], c[sel], 1]
    return rho, u


def compare_runs(ns, field, res, g, K=16, tol=1e-6, check_every=100, max_steps=200_000, infer_s=0.0):
    """Runs one sample from rest and from the predicted field to the residual
    tol; returns steps, seconds (the warm run's include the inference time
    given) and permeabilities."""
    import torch

    b = M.build_stencils_for(ns, K, ns.h)
    perm = b["perm"]
    res_out = {}
    pred = node_fields(ns, res, field)
    for name, init in (("rest", (np.ones(ns.n), np.zeros((ns.n, 2)))), ("warm", pred)):
        sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.FIELDS, storage=M.F32,
                           tau_plus=1.0, g=(g, 0.0), box_area=float(np.prod(ns.hi - ns.lo)))
        sim.init_state(init[0][perm], init[1][perm])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, r, red = sim.run_to_steady(ns.h, tol=tol, check_every=check_every, max_steps=max_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0 + (infer_s if name == "warm" else 0.0)
        k = float(red[M._lib.RED_PERMEABILITY])
        res_out[name] = {"steps": steps, "seconds": dt, "permeability": k, "residual": r}
        if name == "rest":
            # the prediction against the steady state it should have been: its
            # error, the ratio of its flux to the steady flux, and its error
            # once rescaled to the steady flux (the error of its shape)
            _, u_ss, _ = sim.macroscopic(ns.h)
            u_ss = u_ss.cpu().numpy()
            u_p = pred[1][perm]
            fl = ns.kind[perm] == nodesets.FLUID
            a = b["area"][fl]
            ratio = float(np.sum(a * u_p[fl, 0]) / np.sum(a * u_ss[fl, 0]))
            nrm = np.linalg.norm(u_ss[fl])
            res_out["prediction"] = {"rel_err": float(np.linalg.norm(u_p[fl] - u_ss[fl]) / nrm), "flux_ratio": ratio,
                                     "rel_err_flux_matched": float(np.linalg.norm(u_p[fl] / ratio - u_ss[fl]) / nrm)}
        del sim
    return res_out
