"""Launch-shape autotuners: batched runs (tune) and single node sets
(tune_simulation).

Times the batched step (mlbm_step_batched, graph replay, no retirement) on
the actual batch in two stages and keeps the fastest: first the tile size and
the XCD-contiguous chunking, then, with those, the persistent grid together
with the size of the sample groups that run their steps back to back (a group
that fits the memory-side cache is read from it instead of HBM on all but its
first step; a grid at least as large as a group's tile count gives every
workgroup one tile of it).
Results are cached in a JSON file keyed by GPU architecture, stencil size,
variant, storage, and node and sample counts rounded to powers of two, so a
later run on a similar batch reuses them.
"""
from __future__ import annotations

import json
import math
import os

TILES = (64, 128, 256)
XCD = (1, 0)
GRIDS = (1024, 2048, 4096)
GROUP_BYTES = (0.0, 96e6, 160e6, 240e6)
GRID0 = 2048


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "mlbm", "autotune.json")


def cache_key(batch) -> str:
    import torch

    arch = torch.cuda.get_device_properties(batch.sim.state_d[0].device).gcnArchName.split(":")[0]
    p = batch.sim.params
    return (f"{arch}|K{batch.K}|v{p.variant}|s{p.storage}|N2^{round(math.log2(batch.N))}"
            f"|S2^{round(math.log2(len(batch.sizes)))}")


def _time(batch, steps):
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.run(steps, tol=0.0, use_graph=True)
    e1.record(batch.stream)
    batch.stream.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(batch, steps=200, cache_path=None, use_cache=True, rho_u=None):
    """Picks the fastest launch shape for `batch` (a BatchSimulation) and
    applies it.  Returns {"tile", "grid", "xcd", "group_bytes", "ms_per_step",
    "timings", "cached"}.  The batch state is re-initialised (at rest, or from rho_u =
    (rho_list, u_list)) after timing."""
    cache_path = cache_path or default_cache_path()
    key = cache_key(batch)
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if use_cache and key in cache:
        best = dict(cache[key], cached=True)
    else:
        sizes = batch.sizes
        init = rho_u or ([None] * len(sizes), [None] * len(sizes))
        timings = []
        group0 = batch.group_bytes

        def run(tile, xcd, grid, gb):
            batch.set_tile(tile)
            batch.sim.params.xcd_remap = xcd
            batch.batch.grid = grid
            batch.set_groups(gb)
            _reinit(batch, init)
            _time(batch, batch.batch.check_every)  # warm-up (graph build, caches)
            timings.append({"tile": tile, "grid": grid, "xcd": xcd, "group_bytes": gb,
                            "ms_per_step": _time(batch, steps)})

        for tile in TILES:
            for xcd in XCD:
                run(tile, xcd, GRID0, group0)
        first = min(timings, key=lambda r: r["ms_per_step"])
        for grid in GRIDS:
            for gb in GROUP_BYTES:
                if grid != GRID0 or gb != group0:
                    run(first["tile"], first["xcd"], grid, gb)
        best = dict(min(timings, key=lambda r: r["ms_per_step"]))
        best["timings"] = timings
        cache[key] = {k: best[k] for k in ("tile", "grid", "xcd", "group_bytes", "ms_per_step")}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
        best["cached"] = False
    batch.set_tile(best["tile"])
    batch.batch.grid = best["grid"]
    batch.sim.params.xcd_remap = best["xcd"]
    batch.set_groups(best["group_bytes"])
    _reinit(batch, rho_u or ([None] * len(batch.sizes), [None] * len(batch.sizes)))
    return best


def _reinit(batch, rho_u):
    import numpy as np

    rho_list = [np.ones(m) if r is None else r for m, r in zip(batch.sizes, rho_u[0])]
    u_list = [np.zeros((m, 2)) if u is None else u for m, u in zip(batch.sizes, rho_u[1])]
    batch.init_state(rho_list, u_list)


SIM_TILES = (0, 64, 128, 256)
SIM_LANES = (1, 8)
SIM_SWEEPS = (1, 0)


def sim_cache_key(sim) -> str:
    import torch

    arch = torch.cuda.get_device_properties(sim.state_d[0].device).gcnArchName.split(":")[0]
    p = sim.params
    return f"sim2|{arch}|K{sim.K}|v{p.variant}|s{p.storage}|N2^{round(math.log2(sim.n))}"


def tune_simulation(sim, steps=200, cache_path=None, use_cache=True):
    """Picks the mapping (one lane per node, or a group of eight lanes per
    node), tile size (0 = gathers from global memory, else LDS-staged tiles
    of that many nodes), XCD-contiguous tiles and alternating sweeps for a
    Simulation by timing mlbm_step on its own node set, and applies them.
    Shapes the library refuses for this set (eight lanes on hybrid or
    per-departure sets, with 256-node tiles, or for stencil sizes without an
    eight-lane kernel) are skipped.  The state is advanced by the timing runs;
    re-initialise it afterwards.  Returns {"lanes", "tile", "xcd", "sweeps",
    "ms_per_step", "timings", "cached"}."""
    import torch

    from .mlbm import MlbmError

    cache_path = cache_path or default_cache_path()
    key = sim_cache_key(sim)
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if use_cache and key in cache:
        best = dict(cache[key], cached=True)
    else:
        timings = []
        stream = torch.cuda.current_stream()
        for lanes in SIM_LANES:
            sim.params.lanes_per_node = lanes
            for tile in SIM_TILES:
                sim.set_tile(tile)
                for xcd in XCD:
                    for sweeps in SIM_SWEEPS:
                        sim.params.xcd_remap = xcd
                        sim.params.alternate_sweeps = sweeps
                        try:
                            sim.step(steps // 4)
                        except MlbmError as e:
                            if e.code != -5:    # only unsupported shapes are skipped
                                raise
                            continue
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        sim.step(steps)
                        e1.record(stream)
                        e1.synchronize()
                        timings.append({"lanes": lanes, "tile": tile, "xcd": xcd, "sweeps": sweeps,
                                        "ms_per_step": e0.elapsed_time(e1) / steps})
        best = dict(min(timings, key=lambda r: r["ms_per_step"]))
        best["timings"] = timings
        cache[key] = {k: best[k] for k in ("lanes", "tile", "xcd", "sweeps", "ms_per_step")}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
        best["cached"] = False
    sim.params.lanes_per_node = best.get("lanes", 1)
    sim.set_tile(best["tile"])
    sim.params.xcd_remap = best["xcd"]
    sim.params.alternate_sweeps = best["sweeps"]
    return best
