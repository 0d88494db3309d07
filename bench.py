#!/usr/bin/env python3
"""Throughput of the fused meshless LBM step on one MI355X.

Workload (default): the Karman street channel, 22D x 4.1D with a cylinder of
diameter D at (2D, 2D), ~4.9e5 scattered nodes with 4x the density within 1D
of the cylinder, K = 16 nearest-node stencils, streaming-distance scale s = 1
(Re = 100 from a parabolic inflow u_max = 0.05), BGK, FP32 populations.  A
"step" is one time step over every node: the fused gather + collision kernel.

Prints one JSON line: MNUPS (10^6 node updates per second), the HBM roofline
fraction of the step kernel from its algorithmic bytes, and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MNUPS and HBM fraction of fused step; time-to-steady-state plain vs warm-start"


def kernel_source_digest():
    """Digest of what decides the one-lane step kernels' traffic: the device
    code of mlbm_step.hip (everything before its dispatch section),
    mlbm_step's launch logic and the device helpers they include; host-only
    entry points and the eight-lane kernels (a file of their own) do not void
    the stored counters."""
    csrc = os.path.join(ROOT, "paper_2312_14789_amd", "csrc")
    with open(os.path.join(csrc, "mlbm_step.hip")) as f:
        src = f.read()
    device = src[:src.index("// ---- dispatch")]
    a = src.index('extern "C" int mlbm_step(')
    launch = src[a:src.index("\n}\n", a)]
    h = hashlib.sha256()
    h.update(device.encode())
    h.update(launch.encode())
    with open(os.path.join(csrc, "mlbm_device.h")) as f:
        h.update(f.read().encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(f"{kernel}|{workload}")
    if not ent or ent.get("source_digest") != kernel_source_digest():
        return None
    return ent.get("hbm_bytes_per_launch")


def _oracle_stencils(b):
    """The builder's arrays in the oracle's format (source populations from
    the bounce-back bits); the oracle's own builder is not part of the step."""
    import numpy as np

    from oracle import mlbm as omlbm

    src = np.where((b["bb"][:, None] >> np.arange(8)[None, :]) & 1,
                   np.array([3, 4, 1, 2, 7, 8, 5, 6])[None, :], np.arange(1, 9)[None, :])
    return omlbm.Stencils(idx=b["idx"].astype(np.int64), w=b["w"], src=src, point=None, area=b["area"])


def _oracle_steps(ns_perm, st, tau, budget_s):
    """(steps, seconds) of the oracle's population step (collide all nodes,
    then stream all nodes) from rest on all nodes, about budget_s long."""
    import numpy as np

    from oracle import mlbm as omlbm

    n = ns_perm.n
    f = omlbm.init_populations(np.ones(n), np.zeros((n, 2)))
    t0 = time.perf_counter()
    f = omlbm.step(f, ns_perm, st, tau, tau)
    one = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    for _ in range(steps):
        f = omlbm.step(f, ns_perm, st, tau, tau)
    return steps, time.perf_counter() - t0


_FORK_ARGS = None


def _oracle_worker(_):
    ns_perm, st, tau, budget_s = _FORK_ARGS
    return _oracle_steps(ns_perm, st, tau, budget_s)


def cpu_baseline(ns_perm, b, tau, budget_s=15.0, workers=0):
    """The oracle's step on the full node set, timed on the host: one process
    (numpy runs the step on one thread), and, with workers > 1, that many
    forked processes stepping their own copy of the same workload at once
    (all-core throughput: the sum of their rates).  Must run before the
    process touches the GPU (the workers are forked)."""
    global _FORK_ARGS
    import multiprocessing as mp

    n = ns_perm.n
    st = _oracle_stencils(b)
    steps, dt = _oracle_steps(ns_perm, st, tau, budget_s)
    out = {"value": n * steps / dt / 1e6, "unit": "MNUPS", "cores": 1, "kind": "oracle",
           "sample": f"{steps} oracle FP64 steps on all {n} nodes of the same workload "
                     f"({dt:.1f} s, numpy, one thread)"}
    if workers > 1:
        _FORK_ARGS = (ns_perm, st, tau, budget_s)
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_oracle_worker, range(workers))
        _FORK_ARGS = None
        rate = sum(n * k / t for k, t in res) / 1e6
        out["all_cores"] = {"value": rate, "unit": "MNUPS", "cores": workers, "kind": "oracle",
                            "sample": f"{workers} processes, each {min(k for k, _ in res)}-{max(k for k, _ in res)} "
                                      f"oracle FP64 steps on its own copy of all {n} nodes (~{budget_s:g} s each)"}
    return out


def timed_steps(sim, steps, warmup, torch):
    """Average launch time (s) of `steps` steps after `warmup`, HIP events on
    the stream the library launches on."""
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def karman_precision_row(M, units, np, torch, ns, b, tau, tau_m, storage_name, steps=2000, warmup=100):
    """The headline workload with another state storage, e.g. FP64 state,
    weights and arithmetic (the paper's precision: doubles, Sec. 3.2 memory
    model): MNUPS and the HBM fraction from its own algorithmic bytes."""
    storage = getattr(M, storage_name)
    perm = b["perm"]
    sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.POPULATIONS,
                       storage=storage, tau_plus=tau, tau_minus=tau_m, bc=ns.boundary_values()[perm], tile=256)
    sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
    per = timed_steps(sim, steps, warmup, torch)
    _, _, red = sim.macroscopic(1.0, want_fields=False)
    bad = int(red[M._lib.RED_N_BAD].item())
    bpn = units.algorithmic_bytes_per_node(M.POPULATIONS, storage, sim.sizes.k_padded)
    del sim
    return {"storage": storage_name.lower(), "MNUPS": round(ns.n / per / 1e6, 1), "avg_launch_us": round(per * 1e6, 2),
            "steps": steps, "bytes_per_node": bpn, "achieved_GBps": round(bpn * ns.n / per / 1e9, 1),
            "frac": round(bpn * ns.n / per / 1e9 / HBM_PEAK_GBS, 4), "unstable_nodes": bad}


def karman_large_row(M, units, nodesets, np, torch, n_target=2_000_000, steps=2000, warmup=100):
    """The FP32 step on a Karman channel of ~2e6 stratified nodes (same
    geometry and refinement, s = 1), whose per-step traffic (~1.3 GB) is five
    times the 256 MB memory-side cache: its HBM fraction has no help from
    that cache, unlike the ~0.32 GB of the headline set."""
    t0 = time.time()
    ns = nodesets.karman(n_target=n_target, poisson=False)
    dx = units.delta_x(ns.h_min, 1.0)
    tau = units.tau_for_reynolds(0.05, 1.0, dx, 100.0)
    b = M.build_stencils_for(ns, 16, dx)
    perm = b["perm"]
    print(f"# large Karman set: {ns.n} nodes built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.POPULATIONS,
                       storage=M.F32, tau_plus=tau, tau_minus=tau, bc=ns.boundary_values()[perm], tile=256)
    sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
    per = timed_steps(sim, steps, warmup, torch)
    _, _, red = sim.macroscopic(dx, want_fields=False)
    bad = int(red[M._lib.RED_N_BAD].item())
    bpn = units.algorithmic_bytes_per_node(M.POPULATIONS, M.F32, sim.sizes.k_padded)
    del sim
    return {"workload": f"Karman street channel 22Dx4.1D, {ns.n} stratified nodes (4x denser within 1D of the "
                        f"cylinder), K=16, s=1, BGK tau={tau:.4f}, f32 populations",
            "nodes": ns.n, "bytes_per_step": bpn * ns.n, "MNUPS": round(ns.n / per / 1e6, 1),
            "avg_launch_us": round(per * 1e6, 2), "achieved_GBps": round(bpn * ns.n / per / 1e9, 1),
            "frac": round(bpn * ns.n / per / 1e9 / HBM_PEAK_GBS, 4), "unstable_nodes": bad}


def porous_throughput(args, M, units, nodesets, np, torch):
    """MLBM1 (tau = 1, the porous workload's variant) on the 1e6-node porous
    sample: the fused fields step timed like the Karman line, with its
    roofline and, while the kernel source matches, the measured traffic."""
    storage = {"f64": M.F64, "f32": M.F32, "f16s": M.F16S, "bf16": M.BF16}[args.storage]
    ns = nodesets.porous()
    dx = ns.h / args.s
    g = 3.242e-8
    b = M.build_stencils_for(ns, args.K, dx)
    perm = b["perm"]
    sigma = 23 if storage == M.F16S else 0
    sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.FIELDS, storage=storage,
                       tau_plus=1.0, g=(g, 0.0), scale_exp=sigma, tile=args.tile, xcd_remap=args.xcd,
                       alternate_sweeps=args.sweeps, stochastic_rounding=args.sr, weights16=args.weights16)
    n = ns.n
    sim.init_state(np.ones(n), np.zeros((n, 2)))
    sim.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    per_launch_s = ms / 1e3 / args.steps
    _, _, red = sim.macroscopic(dx, want_fields=False)
    bad = int(red.cpu().numpy()[M._lib.RED_N_BAD])
    kp = sim.sizes.k_padded
    bpn = units.algorithmic_bytes_per_node(M.FIELDS, storage, kp, args.weights16)
    achieved = bpn * n / per_launch_s / 1e9
    workload = (f"porous-n{n}-K{args.K}-s{args.s:g}" + ("" if args.storage == "f32" else f"-{args.storage}")
                + ("-w16" if args.weights16 else ""))
    return {"metric": "MNUPS and HBM fraction of the fused MLBM1 step", "value": round(n * args.steps / (ms / 1e3) / 1e6, 1),
            "unit": "MNUPS", "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
            "dtype": args.storage + (" state, f16 weights" if args.weights16 else ""),
            "config": {"workload": f"porous unit box, {n} nodes, phi={ns.fluid_area():.3f}, {len(ns.disks)} disks, "
                                   f"MLBM1 (tau=1), K={args.K}, s={args.s:g}, g_lb={g:g}", "unstable_nodes": bad},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic("k_step_fields_lds", workload),
                         "kernel": "k_step_fields_lds", "bytes_per_node": bpn,
                         "avg_launch_us": round(per_launch_s * 1e6, 2)}}


def copy_calibration():
    """A plain 1 GiB device-to-device copy: the reference that scales the HBM
    byte counters and the practical bandwidth of the box."""
    import torch

    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": ms,
                      "GBps_read_plus_write": 2 * 4 * n / ms / 1e6}), flush=True)
    # a read-only stream of 2 GiB (mlbm_read_probe): the practical bandwidth of
    # a kernel that, like the step, mostly reads
    from paper_2312_14789_amd import probe

    plib = probe.load()
    z = torch.ones(2 * n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for per_thread in (2, 4, 8):
        out = torch.empty(8 * n // (16 * per_thread), dtype=torch.float32, device="cuda")
        call = lambda: probe.read_probe(plib, z.data_ptr(), 8 * n, per_thread, out.data_ptr(),  # noqa: E731
                                        ctypes.c_void_p(stream.cuda_stream))
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(10):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        res[per_thread] = {"ms": ms, "GBps_read": 8 * n / ms / 1e6,
                           "GBps_read_plus_write": (8 * n + 4 * out.numel()) / ms / 1e6}
    print(json.dumps({"read_probe_bytes": 8 * n, "per_thread": res}), flush=True)


def batched_intervals(M, nodesets, np, torch, n_samples=64, tol=1e-6, g=3.242e-8, grid=2048, group_bytes=240e6):
    """The 64-sample batch of the batched workload run 100 steps at a time
    (direct launches, a host synchronisation after each interval), each
    interval timed with its active node count: the throughput of the batched
    kernels while samples retire, by phase."""
    t0 = time.time()
    sets = nodesets.porous_batch(n_samples, n_range=(50_000, 400_000), r_range=(0.01, 0.03))
    built = [M.build_stencils_for(ns, 16, ns.h) for ns in sets]
    print(f"# {n_samples} samples built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    batch = M.BatchSimulation([(b, ns.kind[b["perm"]], None) for b, ns in zip(built, sets)], variant=M.FIELDS,
                              storage=M.F32, tau_plus=1.0, g=(g, 0.0), tile=256, check_every=100, grid=grid,
                              group_bytes=group_bytes)
    sizes = np.array(batch.sizes)

    def rest():
        batch.init_state([np.ones(n) for n in sizes], [np.zeros((n, 2)) for n in sizes])

    rest()
    batch.run(200, tol=0.0, use_graph=False)  # warm-up; tol 0 retires nothing
    rest()
    torch.cuda.synchronize()
    rows = []
    while len(rows) < 1000:
        steps, _, _ = batch.results()
        active = sizes[steps <= 0]
        if active.size == 0:
            break
        t = time.perf_counter()
        batch.run(100, tol=tol, use_graph=False)
        batch.stream.synchronize()
        rows.append((int(active.size), int(active.sum()), time.perf_counter() - t))
        if len(rows) % 50 == 0:
            print(f"# interval {len(rows)}: {active.size} samples active", file=sys.stderr, flush=True)
    n_act = np.array([r[0] for r in rows])
    upd = np.array([r[1] for r in rows], float) * 100
    dt = np.array([r[2] for r in rows])
    phases = {}
    for name, sel in (("all active", n_act == n_samples), ("partly retired", (n_act < n_samples) & (n_act > 4)),
                      ("last 4 or fewer", n_act <= 4)):
        if sel.any():
            phases[name] = {"intervals": int(sel.sum()), "seconds": round(float(dt[sel].sum()), 3),
                            "MNUPS": round(float(upd[sel].sum() / dt[sel].sum() / 1e6), 1)}
    return {"metric": "batched throughput by phase", "workload": f"{n_samples} porous samples, {int(sizes.sum())} "
            f"nodes, MLBM1 FP32, K=16, 100-step intervals without graphs, grid {grid}, groups of "
            f"{group_bytes:g} B", "seconds": round(float(dt.sum()), 3),
            "MNUPS": round(float(upd.sum() / dt.sum() / 1e6), 1), "phases": phases}


def karman_s_sweep(M, units, np, torch, ns, args, storage, tau, tau_m, scales=(2.0, 4.0), steps=50_000):
    """The Karman workload at larger streaming-distance scales s (Re = 100 s at
    fixed tau, Sec. 2.3): `steps` steps from rest on the same node set, each
    checked for unstable nodes, with its throughput."""
    rows = []
    for s_ in scales:
        dx = units.delta_x(ns.h_min, s_)
        b = M.build_stencils_for(ns, args.K, dx, lattice_h=ns.h if args.hybrid else 0.0)
        perm = b["perm"]
        sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.POPULATIONS,
                           storage=storage, tau_plus=tau, tau_minus=tau_m, bc=ns.boundary_values()[perm],
                           tile=args.tile, lagrange=b["lagrange"], w_lagrange=b["w_lagrange"])
        sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, u, red = sim.macroscopic(dx)
        red = red.cpu().numpy()
        bad = int(red[M._lib.RED_N_BAD])
        rows.append({"s": s_, "Re": 100.0 * s_, "dx": dx, "steps": steps, "unstable_nodes": bad,
                     "max_speed": None if bad else float(u.norm(dim=1).max()),
                     "MNUPS": round(ns.n * steps / dt / 1e6, 1)})
        print(f"# s={s_:g}: {steps} steps, {bad} unstable nodes, {rows[-1]['MNUPS']} MNUPS", file=sys.stderr,
              flush=True)
        del sim
    return rows


TTS_RUNS = (("f32", "F32", 0, "field", 200_000), ("f32_mean", "F32", 0, "mean", 200_000),
            ("f16s", "F16S", 0, "field", 60_000), ("f16s_sr_mean", "F16S", 1, "mean", 200_000),
            ("bf16", "BF16", 0, "field", 60_000), ("bf16_sr_mean", "BF16", 1, "mean", 200_000),
            ("f16s_sr_mean_w16", "F16S", 1, "mean", 200_000), ("bf16_sr_mean_w16", "BF16", 1, "mean", 200_000))
TTS_RUNS_INERTIAL = (("f32", "F32", 0, "field", 600_000), ("f32_mean", "F32", 0, "mean", 600_000),
                     ("f16s_sr_mean", "F16S", 1, "mean", 600_000), ("bf16_sr_mean", "BF16", 1, "mean", 600_000),
                     ("f16s_sr_mean_w16", "F16S", 1, "mean", 600_000))


def porous_time_to_steady(M, units, nodesets, np, torch, tol=1e-6, g=3.242e-8, s=1.0, runs=TTS_RUNS):
    """The porous workload (1e6 nodes, phi = 0.7, MLBM1; s = 1: Darcy regime,
    Re ~ 0.1; s = 4: inertial, Re ~ 7) run from rest to steady state with
    FP32, FP16 (scaled offsets) and BF16 state: steps, seconds and
    permeability, the 16-bit permeabilities relative to the FP32 one (the
    first run of `runs` must be FP32; runs named *_w16 read FP16 weights).  Criteria: the field residual between checks
    100 steps apart below tol (FP32; 16-bit rounding keeps the field residual
    near the storage ulp, so 16-bit runs stop at the step cap), and the
    relative change of the mean velocity between checks 1000 steps apart below
    10 tol (all storages; 16-bit with stochastic rounding): the same rate per
    step, measured over an interval long enough that the rounding noise of the
    mean stays below it (the paper's criterion is a rate too, Sec. 3.2)."""
    t0 = time.time()
    ns = nodesets.porous()
    dx = ns.h / s
    b = M.build_stencils_for(ns, 16, dx)
    perm = b["perm"]
    nu = units.nu_lattice(1.0)
    out = {"workload": f"porous unit box, {ns.n} nodes, phi={ns.fluid_area():.3f}, {len(ns.disks)} disks, "
                       f"MLBM1 (tau=1), K=16, s={s:g}, g_lb={g:g}", "tol": tol,
           "setup_s": None, "runs": {}}
    k_ref = None
    sigma = 0
    for name, storage_name, sr, crit, cap in runs:
        storage = getattr(M, storage_name)
        sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.FIELDS,
                           storage=storage, tau_plus=1.0, g=(g, 0.0), scale_exp=sigma, stochastic_rounding=sr,
                           weights16=name.endswith("_w16"), box_area=float(np.prod(ns.hi - ns.lo)))
        if out["setup_s"] is None:
            out["setup_s"] = round(time.time() - t0, 2)
        sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        every, tol_c = (1000, 10.0 * tol) if crit == "mean" else (100, tol)
        steps, res, red = sim.run_to_steady(dx, tol=tol_c, check_every=every, max_steps=cap, criterion=crit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        k = float(red[M._lib.RED_PERMEABILITY])
        umean = red[M._lib.RED_INT_UX] / ns.fluid_area()
        rec = {"criterion": crit, "check_every": every, "tol": tol_c, "stochastic_rounding": sr,
               "weights": "f16" if name.endswith("_w16") else ("f32" if storage != M.F64 else "f64"), "steps": steps,
               "converged": bool(res < tol_c),
               "seconds": round(dt, 3), "residual": res, "permeability": k,
               "Re": umean / dx / nu, "MNUPS": round(ns.n * steps / dt / 1e6, 1)}
        if name == "f32":
            k_ref = k
            _, u, _ = sim.macroscopic(dx)
            sigma = units.f16_scale_exp(float(u.abs().max()))
        else:
            rec["scale_exp"] = sigma if storage == M.F16S else None
            rec["permeability_rel_err_vs_f32"] = abs(k / k_ref - 1.0)
        out["runs"][name] = rec
        print(f"# steady s={s:g} {name}: {steps} steps, {dt:.2f} s, residual {res:.2e}", file=sys.stderr,
              flush=True)
        del sim
    return out


def batched_workload(M, units, nodesets, np, torch, n_samples=64, tol=1e-6, g=3.242e-8, sequential=True,
                     n_range=(50_000, 400_000), r_range=(0.01, 0.03)):
    """64 porous samples (nodes U(5e4, 4e5), porosity U(0.55, 0.85)), MLBM1
    FP32, s = 1, run from rest to a residual of tol in one batched launch
    (persistent tile queue, graph replay, autotuned shape), against the same
    samples run one after another.  A second call with many small samples
    (each too small to fill the GPU alone, with disks of radius 0.05-0.12 so
    that their coarser nodes still resolve them) shows what batching buys
    there."""
    from paper_2312_14789_amd import autotune

    t0 = time.time()
    sets = nodesets.porous_batch(n_samples, n_range=n_range, r_range=r_range,
                                 log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    print(f"# {n_samples} porous samples generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    built = []
    for si, ns in enumerate(sets):
        built.append(M.build_stencils_for(ns, 16, ns.h))
        if si % 32 == 31:
            print(f"# stencils {si + 1}/{n_samples}", file=sys.stderr, flush=True)
    batch = M.BatchSimulation([(b, ns.kind[b["perm"]], None) for b, ns in zip(built, sets)], variant=M.FIELDS,
                              storage=M.F32, tau_plus=1.0, g=(g, 0.0), tile=256, check_every=100)
    setup = time.time() - t0
    print(f"# batched setup {setup:.1f} s, {batch.N} nodes incl. padding", file=sys.stderr, flush=True)
    t1 = time.time()
    best = autotune.tune(batch, steps=200)
    tune_s = time.time() - t1
    print(f"# autotuned in {tune_s:.1f} s: {best['tile']} {best['grid']} {best['xcd']} {best['group_bytes']}",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ran = batch.run(400_000, tol=tol, use_graph=True)
    dt = time.perf_counter() - t2
    steps, res, ux = batch.results()
    sizes = np.array(batch.sizes)
    updates = float(np.sum(sizes * np.abs(steps)))
    out = {"metric": "batched time to steady state", "workload": f"{n_samples} porous samples, "
           f"{int(sizes.sum())} nodes (min {sizes.min()}, max {sizes.max()}), MLBM1 FP32, K=16, s=1, g_lb={g:g}, "
           f"residual {tol:g}", "seconds": round(dt, 3), "steps_run": ran,
           "sample_steps_min_max": [int(steps.min()), int(steps.max())], "unconverged": int(np.sum(steps <= 0)),
           "MNUPS_effective": round(updates / dt / 1e6, 1), "setup_s": round(setup, 1),
           "groups": int(batch.batch.n_groups),
           "autotune": {k: best[k] for k in ("tile", "grid", "xcd", "group_bytes", "ms_per_step", "cached")},
           "autotune_s": round(tune_s, 1)}
    if sequential:
        # the same samples one after another, each in its own launches (time
        # of the stepping loops only, no construction or upload)
        tile = best["tile"]
        del batch
        seq_seconds = 0.0
        seq_steps = []
        print(f"# batched run {dt:.2f} s; sequential runs follow", file=sys.stderr, flush=True)
        for si, (b, ns) in enumerate(zip(built, sets)):
            if si % 16 == 15:
                print(f"# sequential {si + 1}/{len(sets)}", file=sys.stderr, flush=True)
            sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[b["perm"]], b["area"], variant=M.FIELDS,
                               storage=M.F32, tau_plus=1.0, g=(g, 0.0), tile=tile)
            sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
            torch.cuda.synchronize()
            ta = time.perf_counter()
            st_, _, _ = sim.run_to_steady(ns.h, tol=tol, check_every=100, max_steps=400_000)
            torch.cuda.synchronize()
            seq_seconds += time.perf_counter() - ta
            seq_steps.append(st_)
            del sim
        out["sequential"] = {"seconds": round(seq_seconds, 3),
                             "speedup_batched": round(seq_seconds / dt, 3),
                             "same_steps_per_sample": bool(np.array_equal(np.array(seq_steps), steps))}
    return out


def darcy_workload(M, units, nodesets, np, torch, g_lb=1e-7, max_steps=1_560_000, tol=1e-6, K=25):
    """Onset of inertia in the porous sample of Sec. 3.2: MLBM1 (tau = 1) on
    the hybrid porous channel at a fixed lattice forcing g_lb for a sweep of
    streaming distances dx, all of them in one batched launch (one sample per
    dx).  With the physical viscosity 1 (dt = nu_lb dx^2), each dx gives the
    physical acceleration g = g_lb dx / dt^2, the mean velocity <u> (Eq. 23),
    Re = <u> (unit length and viscosity) and the tortuosity
    T_V = <|u|> / <u> (Eq. 25), at steady state or at the step cap."""
    t0 = time.time()
    ns = nodesets.porous_channel()
    dxs = [2e-3, 1.35e-3, 1.05e-3, 7.5e-4, 6e-4, 4.5e-4, 2.7e-4, 2.1e-4, 1.5e-4]  # Sec. 3.2's sweep
    built = [M.build_stencils_for(ns, K, dx, lattice_h=ns.h) for dx in dxs]
    batch = M.BatchSimulation([(b, ns.kind[b["perm"]], None) for b in built], variant=M.FIELDS, storage=M.F32,
                              tau_plus=1.0, g=(g_lb, 0.0), tile=256, check_every=100)
    batch.init_state([np.ones(ns.n)] * len(dxs), [np.zeros((ns.n, 2))] * len(dxs))
    setup = time.time() - t0
    print(f"# darcy sweep: {len(dxs)} samples of {ns.n} nodes, setup {setup:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ran = 0
    while ran < max_steps:  # in slices, so progress shows
        ran += batch.run(min(100_000, max_steps - ran), tol=tol, use_graph=True)
        steps_now, _, _ = batch.results()
        print(f"# {ran} steps, {int(np.sum(steps_now == 0))} samples running", file=sys.stderr, flush=True)
        if not np.any(steps_now == 0):
            break
    torch.cuda.synchronize()
    dt_run = time.perf_counter() - t1
    steps, res, _ = batch.results()
    _, u, _ = batch.sim.macroscopic(1.0)
    u = u.cpu().numpy()
    phi = ns.fluid_area()
    nu_lb = units.nu_lattice(1.0)
    rows = []
    for s_, (dx, b) in enumerate(zip(dxs, built)):
        o, m = int(batch.node_off[s_]), batch.sizes[s_]
        us = u[o:o + m]
        area = b["area"]
        int_ux = float(np.sum(area * us[:, 0]))
        int_speed = float(np.sum(area * np.hypot(us[:, 0], us[:, 1])))
        dt = units.time_step(dx, 1.0, 1.0)
        u_mean = int_ux / phi * dx / dt
        rows.append({"dx": dx, "s_bulk": round(ns.h / dx, 3), "g": units.acceleration_phys(g_lb, dx, dt),
                     "u_mean": u_mean, "Re": u_mean, "T_V": int_speed / int_ux if int_ux else None,
                     "steps": int(abs(steps[s_])) if steps[s_] else ran, "converged": bool(steps[s_] > 0),
                     "unstable": bool(steps[s_] < 0), "residual": float(res[s_])})
    # Darcy: <u> proportional to g; the deviation is <u>/g relative to the smallest g
    base = rows[0]["u_mean"] / rows[0]["g"]
    for r in rows:
        r["darcy_ratio"] = r["u_mean"] / r["g"] / base
    return {"metric": "Darcy deviation and tortuosity versus Re (MLBM1, batched sweep over dx)",
            "workload": f"porous channel (Sec. 3.2 arrangement): {ns.n} nodes, phi={phi:.3f}, {len(ns.disks)} disks, "
                        f"periodic x, no-slip walls y, hybrid lattice h={ns.h:g} / band nodes to h={ns.h_min:g}; "
                        f"g_lb={g_lb:g}, K={K}, residual {tol:g} or {max_steps} steps",
            "seconds": round(dt_run, 2), "steps_run": ran, "setup_s": round(setup, 1),
            "MNUPS_effective": round(sum(r["steps"] for r in rows) * ns.n / dt_run / 1e6, 1) if dt_run else None,
            "rows": rows}


def strouhal_from_lift(lift, every, d_lattice, u0, hysteresis=0.5):
    """St = f d / U0 from a lift series sampled every `every` steps (after
    the transient), in lattice units (f in cycles per step, d in streaming
    distances).  Returns (St from the mean period between the first and last
    upward crossings of the mean-free signal; St from the peak of its
    Hann-windowed spectrum, zero-padded 8x).  An upward crossing counts once
    the signal has risen from below -theta to above +theta (theta =
    `hysteresis` x its RMS), so noise near zero adds no crossings; its time is
    the last sign change inside that rise, linearly interpolated between
    samples.  NaN if there are fewer than three crossings."""
    import numpy as np

    tail = np.asarray(lift, dtype=np.float64)
    tail = tail - tail.mean()
    spec = np.abs(np.fft.rfft(tail * np.hanning(len(tail)), n=8 * len(tail)))
    freqs = np.fft.rfftfreq(8 * len(tail), d=every)
    st_fft = freqs[int(np.argmax(spec[1:]) + 1)] * d_lattice / u0
    theta = hysteresis * float(np.sqrt(np.mean(tail * tail)))
    crossings = []
    low, last_up = False, None
    for j in range(len(tail)):
        if tail[j] < -theta:
            low, last_up = True, None
        elif low and j > 0 and tail[j - 1] < 0.0 <= tail[j]:
            last_up = j - 1
        if low and tail[j] > theta and last_up is not None:
            i = last_up
            crossings.append(i + (-tail[i]) / (tail[i + 1] - tail[i]))
            low = False
    if len(crossings) < 3:
        return float("nan"), float(st_fft)
    period_steps = (crossings[-1] - crossings[0]) / (len(crossings) - 1) * every
    return float(d_lattice / (period_steps * u0)), float(st_fft)


ST_CASES = (("coarsened", "shared", (105, 126, 147, 168)),
            ("coarsened", "shared", (105, 126, 147, 168), 32),
            ("uniform", "shared", (105, 126, 147, 168)),
            ("scattered", "shared", (105, 168)),
            ("coarsened", "per-departure", (105, 168)))


def strouhal_workload(M, units, nodesets, np, torch, cases=ST_CASES, periods=10, transient=10, every=50,
                      dump=None):
    """The paper's cylinder flow (Sec. 3.1): 3 x 1 channel, d = 0.14,
    U0 = 0.01, TRT with tau+ = 0.53 and Lambda = 3/16, K = 25 stencils,
    biquadratic Lagrange on the lattice part, simple bounce-back on the
    cylinder; Re = U0 d / nu raised by shrinking dx (Sec. 2.3).  The lift
    (momentum exchange on the cylinder) is sampled every `every` steps; after
    `transient` shedding periods (estimated with St = 0.2) the next `periods`
    give St = f d / U0 (lattice units: f in cycles per step, d in streaming
    distances), f from the mean spacing of upward zero crossings (the peak of
    the zero-padded spectrum as a check).  Each case names the node set
    ("coarsened": h 1/200 on the cylinder to 1/25, the set the paper measures
    St on; "uniform": 1/200 everywhere, scattered only near the cylinder and
    its wake; "scattered": 1/200 everywhere, all scattered: the paper's three
    timing scenarios), the stencil form ("per-departure":
    the K nearest nodes of each departure point, as the paper states;
    "shared": one stencil per node for its eight departure points), the
    Reynolds numbers and optionally the stencil size (default 25)."""
    names = {c[0] for c in cases}
    recipes = {"coarsened": {}, "uniform": dict(h_max=1.0 / 200, grade=0.15, wake_stretch=0.3),
               "scattered": dict(h_max=1.0 / 200, grade=10.0, wake_stretch=1.0)}
    sets = {k: nodesets.karman_paper(**v) for k, v in recipes.items() if k in names}
    d, u0, tau = 0.14, 1e-2, 0.53
    tau_m = 0.5 + (3.0 / 16.0) / (tau - 0.5)
    nu_lb = units.nu_lattice(tau)
    rows = []
    series = {}
    for case in cases:
        set_name, mode, reynolds = case[:3]
        K = case[3] if len(case) > 3 else 25
        ns = sets[set_name]
        for re in reynolds:
            dx = u0 * d / (re * nu_lb)
            b = M.build_stencils_for(ns, K, dx, lattice_h=ns.h, per_departure=mode == "per-departure",
                                     simple_bounce_back=True)
            perm = b["perm"]
            # per-departure rows of block centres carry their block weights
            # themselves; shared stencils take the one block table
            lag = dict(lagrange=b["lagrange"], w_lagrange=b["w_lagrange"]) if mode == "shared" else {}
            sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.POPULATIONS,
                               storage=M.F32, tau_plus=tau, tau_minus=tau_m, bc=ns.boundary_values()[perm],
                               tile=256, graph_steps=every, **lag)
            # at rest, boundary values on the Dirichlet nodes, and a small transverse
            # kick behind the cylinder so the shedding does not wait for round-off
            xy = ns.xy[perm]
            u = np.zeros((ns.n, 2))
            wake = (xy[:, 0] > 0.6) & (xy[:, 0] < 1.0) & (np.abs(xy[:, 1] - 0.5) < 0.1)
            u[wake, 1] = 0.1 * u0
            dmask = ns.kind[perm] == nodesets.DIRICHLET
            u[dmask] = ns.boundary_values()[perm][dmask, 1:3]
            sim.init_state(np.ones(ns.n), u)
            t_shed = (d / dx) / (0.2 * u0)  # steps per period for St ~ 0.2
            n_samples = int((transient + periods) * t_shed / every)
            lift = np.zeros(n_samples)
            stream = torch.cuda.Stream()     # graph replay needs a stream of its own
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s_ in range(n_samples):
                sim.step(every, stream=stream)
                _, _, red = sim.macroscopic(dx, want_fields=False, stream=stream)
                stream.synchronize()
                lift[s_] = float(red[M._lib.RED_FORCE_Y].item())
                if s_ % 4000 == 3999:
                    print(f"# {set_name} {mode} Re {re}: {s_ + 1}/{n_samples} lift samples", file=sys.stderr,
                          flush=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            _, _, red = sim.macroscopic(dx, want_fields=False)
            bad = int(red[M._lib.RED_N_BAD].item())
            tail = lift[int(transient * t_shed / every):]
            st, st_fft = strouhal_from_lift(tail, every, d / dx, u0)
            tail = tail - tail.mean()
            n_steps = n_samples * every
            series[f"{set_name}_{mode}_K{K}_Re{re}"] = lift
            rows.append({"nodes": set_name, "n": ns.n, "block_centres": int(b["n_lagrange"]), "stencils": mode, "K": K,
                         "Re": re, "dx": dx, "s_min": round(ns.h_min / dx, 3), "s_max": round(ns.h / dx, 3),
                         "steps": n_steps, "St": round(float(st), 4), "St_fft": round(float(st_fft), 4),
                         "lift_amplitude": float(np.abs(tail).max()), "lift_rms": float(np.sqrt(np.mean(tail ** 2))),
                         "unstable_nodes": bad, "seconds": round(dt, 2),
                         "ms_per_1000_steps": round(dt / n_steps * 1e6, 2),
                         "MNUPS": round(ns.n * n_steps / dt / 1e6, 1)})
            print(f"# {set_name} {mode} Re {re}: St {st:.4f}, {dt:.1f} s, unstable nodes {bad}", file=sys.stderr,
                  flush=True)
            del sim
    if dump:
        np.savez(dump, every=every, **series)
    return {"metric": "Strouhal number of the cylinder wake vs Re (the paper's configuration)",
            "workload": "3x1 channel, d=0.14, U0=0.01, symmetric node sets "
                        + ", ".join(f"{k}: {v.n} nodes (h {v.h_min:g}..{v.h:g})" for k, v in sets.items())
                        + ", TRT tau+=0.53 Lambda=3/16, K per row (25 by default), simple bounce-back, FP32, lift every "
                        + f"{every} steps, {transient} + {periods} periods",
            "rows": rows}


WS_RES, WS_G = 256, 1e-5
# warm-start leg of the default line: training media, held-out media, epochs
# (the full workload, --workload warmstart, trains on 2000 media for 20 epochs
# and compares on 200)
WS_BENCH = (512, 32, 16)


def warmstart_geometries(n):
    """n random-disk media on 256^2 rasters (16 host worker processes);
    returns (geometries, seconds)."""
    from paper_2312_14789_amd import warmstart

    t0 = time.time()
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)  # noqa: E731
    geoms = warmstart.make_geometries(n, res=WS_RES, workers=16, log=log)
    dt = time.time() - t0
    print(f"# {len(geoms)} warm-start geometries in {dt:.1f} s", file=sys.stderr, flush=True)
    return geoms, dt


def warmstart_workload(np, torch, n_train, n_test, epochs, save="", geoms=None):
    """Learned warm start (network of 5 levels, 32-256 channels, 256^2 rasters):
    train on steady states of random-disk media computed by batched library
    runs, then compare steps and wall time to a residual of 1e-6 from rest and
    from the network's prediction on held-out samples.  geoms: the media, made
    beforehand by warmstart_geometries (before the process touches the GPU,
    since making them forks worker processes)."""
    from paper_2312_14789_amd import unet, warmstart

    res, g = WS_RES, WS_G
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)  # noqa: E731
    t_geo = 0.0
    if geoms is None:
        geoms, t_geo = warmstart_geometries(n_train + n_test)
    train_g, test_g = geoms[:n_train], geoms[n_train:n_train + n_test]
    t0 = time.time()
    fields, steps = warmstart.steady_states(train_g, g, batch_size=64, log=log)
    t_data = time.time() - t0
    train_g, fields, steps, dropped = warmstart.converged_only(train_g, fields, steps)
    print(f"# steady states in {t_data:.1f} s, steps {min(steps)}..{max(steps)}, {dropped} not converged (dropped)",
          file=sys.stderr, flush=True)
    data = warmstart.Dataset(train_g, fields, res)
    del fields
    net = unet.UNet((32, 64, 128, 256, 256), res=res, batch=16, seed=1)
    t0 = time.time()
    hist = warmstart.train(net, data, epochs=epochs, lr=1e-3, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    iters = epochs * (data.n // net.batch)
    # inference time per sample (one batch of 16)
    masks = [m for _, m in test_g]
    warmstart.predict(net, data, masks[:16], data.u_scale, data.r_scale)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    preds = warmstart.predict(net, data, masks, data.u_scale, data.r_scale)
    torch.cuda.synchronize()
    infer = (time.perf_counter() - t0) / len(masks)
    rows = []
    for i, ((ns, _), f) in enumerate(zip(test_g, preds)):
        rows.append(warmstart.compare_runs(ns, f, res, g, infer_s=infer))
        if (i + 1) % 20 == 0:
            log(f"{i + 1}/{len(test_g)} held-out comparisons")
    rest_steps = np.array([r["rest"]["steps"] for r in rows])
    warm_steps = np.array([r["warm"]["steps"] for r in rows])
    rest_s = np.array([r["rest"]["seconds"] for r in rows])
    warm_s = np.array([r["warm"]["seconds"] for r in rows])
    kerr = np.array([abs(r["warm"]["permeability"] / r["rest"]["permeability"] - 1) for r in rows])
    pe = np.array([r["prediction"]["rel_err"] for r in rows])
    pf = np.array([r["prediction"]["flux_ratio"] for r in rows])
    ps = np.array([r["prediction"]["rel_err_flux_matched"] for r in rows])
    if save:
        np.savez(save, **net.state_dict())
    fl = 0.0
    for name, k, ci, co in net.shapes:
        fl += 2.0 * k * k * ci * co * (res >> (int(name[3]) if name != "head" else 0)) ** 2
    return {"metric": "time-to-steady-state plain vs warm-start",
            "workload": f"{len(train_g)} training + {len(test_g)} held-out random-disk media, {res}^2 rasters, "
                        f"MLBM1 FP32 K=16 s=1 g_lb={g:g}, residual 1e-6",
            "steps_rest_mean": float(rest_steps.mean()), "steps_warm_mean": float(warm_steps.mean()),
            "step_ratio_rest_over_warm": float((rest_steps / warm_steps).mean()),
            "seconds_rest_mean": float(rest_s.mean()), "seconds_warm_mean_incl_inference": float(warm_s.mean()),
            "inference_ms_per_sample": round(1e3 * infer, 3),
            "permeability_rel_err_max": float(kerr.max()), "permeability_within_0.5pct": bool(kerr.max() <= 5e-3),
            "prediction": {"rel_err_mean": float(pe.mean()), "flux_ratio_mean": float(pf.mean()),
                           "flux_ratio_abs_dev_mean": float(np.abs(pf - 1).mean()),
                           "rel_err_flux_matched_mean": float(ps.mean())},
            "steps_saved_mean": float((rest_steps - warm_steps).mean()),
            "seconds_saved_mean": float((rest_s - warm_s).mean()),
            "train": {"epochs": epochs, "loss_first": hist[0], "loss_last": hist[-1], "seconds": round(t_train, 1),
                      "iters": iters, "ms_per_iter": round(1e3 * t_train / max(iters, 1), 2),
                      "tflops_fwd_bwd": round(3 * fl * net.batch * iters / t_train / 1e12, 2)},
            "data": {"geometry_s": round(t_geo, 1), "steady_states_s": round(t_data, 1),
                     "steps_min_max": [int(min(steps)), int(max(steps))], "unconverged_dropped": dropped}}


def mapping_workload(M, nodesets, np, torch, sides=(64, 128, 256, 512), steps=2000, warmup=200):
    """One lane per node against a group of eight lanes per node, over node
    sets from 4 096 to 262 144 nodes (periodic jittered grids, K = 16,
    s = 1.5, FP32): microseconds per step of every launch shape (tile 0 =
    global gathers, else LDS tiles of that many nodes), steps replayed as
    graphs of 100 so launch overhead does not hide the kernels.  Population
    form (BGK tau = 0.8) and fields form (tau = 1)."""
    shapes = [(1, 0), (1, 64), (1, 128), (1, 256), (8, 0), (8, 64), (8, 128)]
    rows = []
    stream = torch.cuda.Stream()
    for side in sides:
        ns = nodesets.jittered_grid(side, seed=11)
        dx = 1.0 / side / 1.5
        b = M.build_stencils_for(ns, 16, dx)
        perm = b["perm"]
        rho0, u0 = nodesets.smooth_fields(ns.xy[perm], 3, amp_u=0.01, amp_rho=0.001)
        for variant, tau in ((M.POPULATIONS, 0.8), (M.FIELDS, 1.0)):
            row = {"nodes": ns.n, "variant": "populations" if variant == M.POPULATIONS else "fields", "us_per_step": {}}
            for lanes, tile in shapes:
                sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=variant,
                                   storage=M.F32, tau_plus=tau, tile=tile, lanes_per_node=lanes, graph_steps=100)
                sim.init_state(rho0, u0)
                sim.step(warmup, stream=stream)
                stream.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sim.step(steps, stream=stream)
                e1.record(stream)
                e1.synchronize()
                row["us_per_step"][f"lanes{lanes}-tile{tile}"] = round(e0.elapsed_time(e1) * 1e3 / steps, 2)
                del sim
            best1 = min((v, k) for k, v in row["us_per_step"].items() if k.startswith("lanes1"))
            best8 = min((v, k) for k, v in row["us_per_step"].items() if k.startswith("lanes8"))
            row["best_one_lane"] = best1[1]
            row["best_eight_lanes"] = best8[1]
            row["speedup_eight_lanes"] = round(best1[0] / best8[0], 3)
            row["MNUPS_best"] = round(ns.n / min(best1[0], best8[0]), 1)
            print(f"# {ns.n} nodes {row['variant']}: one lane {best1[0]} us ({best1[1]}), eight lanes "
                  f"{best8[0]} us ({best8[1]})", file=sys.stderr, flush=True)
            rows.append(row)
    # the paper's coarsened cylinder channel: a hybrid set (block centres and
    # scattered nodes in one launch), K = 25, TRT, Re 105 (the Strouhal set)
    ns = nodesets.karman_paper()
    tau = 0.53
    tau_m = 0.5 + (3.0 / 16.0) / (tau - 0.5)
    dx = 1e-2 * 0.14 / (105.0 * (tau - 0.5) / 3.0)
    b = M.build_stencils_for(ns, 25, dx, lattice_h=ns.h, simple_bounce_back=True)
    perm = b["perm"]
    row = {"nodes": ns.n, "variant": "populations, hybrid cylinder channel (K=25, TRT)", "us_per_step": {}}
    for lanes, tile in [(1, 64), (1, 128), (1, 256), (8, 64), (8, 128)]:
        sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.POPULATIONS, storage=M.F32,
                           tau_plus=tau, tau_minus=tau_m, bc=ns.boundary_values()[perm], tile=tile,
                           lagrange=b["lagrange"], w_lagrange=b["w_lagrange"], lanes_per_node=lanes, graph_steps=100)
        sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
        sim.step(warmup, stream=stream)
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps, stream=stream)
        e1.record(stream)
        e1.synchronize()
        row["us_per_step"][f"lanes{lanes}-tile{tile}"] = round(e0.elapsed_time(e1) * 1e3 / steps, 2)
        del sim
    best1 = min((v, k) for k, v in row["us_per_step"].items() if k.startswith("lanes1"))
    best8 = min((v, k) for k, v in row["us_per_step"].items() if k.startswith("lanes8"))
    row.update(best_one_lane=best1[1], best_eight_lanes=best8[1], speedup_eight_lanes=round(best1[0] / best8[0], 3),
               block_centres=int(b["n_lagrange"]))
    print(f"# {ns.n} nodes hybrid cylinder channel: one lane {best1[0]} us ({best1[1]}), eight lanes "
          f"{best8[0]} us ({best8[1]})", file=sys.stderr, flush=True)
    rows.append(row)
    return {"metric": "step time, one lane vs eight lanes per node",
            "workload": "periodic jittered grids (jitter 0.3 h), K=16, s=1.5, FP32, graph replay of 100 steps; "
                        "the paper's coarsened cylinder channel (hybrid, K=25, TRT, Re 105)",
            "rows": rows}


def unet_workload(np, torch, steps=20, warmup=3):
    """The warm-start network's own throughput at its training shape (5
    levels, 32-256 channels, 256^2 rasters, batch 16) on synthetic masks:
    milliseconds and TFLOP/s of a training iteration (forward, loss,
    backward, Adam) and of a forward pass, against the 2.5 PFLOP/s dense bf16
    peak.  FLOPs: 2 k^2 c_in c_out per output pixel per convolution; a
    training iteration counts three such products (forward, data gradient,
    weight gradient)."""
    from paper_2312_14789_amd import unet

    res, B = 256, 16
    net = unet.UNet((32, 64, 128, 256, 256), res=res, batch=B, seed=1)
    rng = np.random.default_rng(0)
    x = torch.zeros((B, res, res, unet.PAD), dtype=torch.bfloat16, device="cuda")
    fluid = (rng.uniform(size=(B, res, res)) > 0.3).astype(np.float32)
    x[..., 0] = torch.from_numpy(fluid).cuda().to(torch.bfloat16)
    xi = x.view(torch.int16)
    target = torch.from_numpy(rng.normal(size=(B, res, res, 3)).astype(np.float32)).cuda()
    mask = torch.from_numpy(fluid).cuda()

    def iteration():
        net.forward(xi)
        net.loss_and_grad(target, mask)
        net.backward()
        net.adam_step(1e-4)

    fl = 0.0
    for name, k, ci, co in net.shapes:
        R = res >> (int(name[3]) if name != "head" else 0)
        fl += 2.0 * k * k * ci * co * R * R * B
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        iteration()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        iteration()
    e1.record(stream)
    torch.cuda.synchronize()
    t_it = e0.elapsed_time(e1) / 1e3 / steps
    e0.record(stream)
    for _ in range(steps):
        net.forward(xi)
    e1.record(stream)
    torch.cuda.synchronize()
    t_fw = e0.elapsed_time(e1) / 1e3 / steps
    return {"metric": "warm-start network throughput (bf16 MFMA, FP32 accumulation)",
            "workload": f"5-level encoder-decoder (32-256 channels), {res}^2 rasters, batch {B}, synthetic masks",
            "train_ms_per_iter": round(t_it * 1e3, 3), "train_TFLOPs": round(3 * fl / t_it / 1e12, 1),
            "forward_ms": round(t_fw * 1e3, 3), "forward_TFLOPs": round(fl / t_fw / 1e12, 1),
            "inference_ms_per_sample": round(t_fw / B * 1e3, 4), "gflop_forward": round(fl / 1e9, 1),
            "peak_TFLOPs_bf16": 2500.0, "frac_train": round(3 * fl / t_it / 1e12 / 2500.0, 4),
            "frac_forward": round(fl / t_fw / 1e12 / 2500.0, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--s", type=float, default=1.0, help="streaming-distance scale (dx = h_min/s)")
    ap.add_argument("--K", type=int, default=16)
    ap.add_argument("--trt", type=int, default=0, help="TRT with Lambda = 3/16 instead of BGK")
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16s", "bf16"])
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--tile", type=int, default=256, help="LDS-staged tile size (0 = global gathers)")
    ap.add_argument("--xcd", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=1, help="alternate the tile sweep direction")
    ap.add_argument("--cached", type=int, default=0, help="ordinary (not non-temporal) weight loads")
    ap.add_argument("--nodes", type=int, default=500_000, help="target node count of the workload")
    ap.add_argument("--hybrid-launches", type=int, default=0, choices=(0, 2),
                    help="hybrid set: 0 = one launch per step for both node kinds, 2 = one launch per kind")
    ap.add_argument("--hybrid", action="store_true",
                    help="hybrid node set: square lattice away from the cylinder and its wake, biquadratic "
                         "Lagrange weights at the block centres")
    ap.add_argument("--stratified", action="store_true",
                    help="Karman nodes by stratified (jittered) samples instead of Poisson-disk fronts")
    ap.add_argument("--no-s-sweep", action="store_true", help="skip the s = 2, 4 stability runs")
    ap.add_argument("--weights16", type=int, default=0, help="FP16 weights (with --storage f16s or bf16)")
    ap.add_argument("--sr", type=int, default=0, help="stochastic rounding of 16-bit stores")
    ap.add_argument("--reorder", type=int, default=1, choices=[0, 1, 2],
                    help="node order: 0 as generated, 1 Morton, 2 reverse Cuthill-McKee")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-steady", action="store_true", help="skip the porous time-to-steady section")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the warm-start leg (steps and seconds to steady state, plain vs warm-start)")
    ap.add_argument("--no-extra-rows", action="store_true",
                    help="skip the FP64 row and the large (beyond the memory-side cache) Karman set")
    ap.add_argument("--st-dump", default=None, help="strouhal: save the lift series (npz) to this path")
    ap.add_argument("--workload", default="karman",
                    choices=["karman", "porous", "batched", "batched-intervals", "warmstart", "darcy", "strouhal",
                             "unet", "mapping"],
                    help="karman: the fused-step throughput line; porous: the MLBM1 step on the 1e6-node "
                         "porous sample; batched: 64 porous samples to steady "
                         "state; batched-intervals: the same batch timed per 100-step interval, by phase; "
                         "warmstart: train the warm-start network and compare time to steady state; "
                         "darcy: mean velocity and tortuosity of the porous channel over a sweep of dx; "
                         "strouhal: the paper's cylinder channel, St from the lift over Re 105-168; "
                         "unet: training and inference throughput of the warm-start network; "
                         "mapping: one against eight lanes per node over node sets of 4k-262k nodes")
    ap.add_argument("--ws-train", type=int, default=2000)
    ap.add_argument("--ws-test", type=int, default=200)
    ap.add_argument("--ws-epochs", type=int, default=20)
    ap.add_argument("--ws-save", default="", help="write the trained warm-start network's weights here (.npz)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a 1 GiB device copy (reference for byte counters and bandwidth)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "halo-exchange design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import nodesets
    from paper_2312_14789_amd import mlbm as M
    from paper_2312_14789_amd import units

    if args.workload == "batched":
        out = batched_workload(M, units, nodesets, np, torch)
        out["small_samples"] = batched_workload(M, units, nodesets, np, torch, n_samples=256,
                                                n_range=(2_000, 20_000), r_range=(0.05, 0.12))
        print(json.dumps(out), flush=True)
        return
    if args.workload == "batched-intervals":
        print(json.dumps(batched_intervals(M, nodesets, np, torch)), flush=True)
        return
    if args.workload == "warmstart":
        print(json.dumps(warmstart_workload(np, torch, args.ws_train, args.ws_test, args.ws_epochs, save=args.ws_save)),
              flush=True)
        return
    if args.workload == "mapping":
        print(json.dumps(mapping_workload(M, nodesets, np, torch)), flush=True)
        return
    if args.workload == "unet":
        print(json.dumps(unet_workload(np, torch, steps=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.workload == "porous":
        print(json.dumps(porous_throughput(args, M, units, nodesets, np, torch)), flush=True)
        return
    if args.workload == "darcy":
        print(json.dumps(darcy_workload(M, units, nodesets, np, torch)), flush=True)
        return
    if args.workload == "strouhal":
        print(json.dumps(strouhal_workload(M, units, nodesets, np, torch, dump=args.st_dump)), flush=True)
        return

    storage = {"f64": M.F64, "f32": M.F32, "f16s": M.F16S, "bf16": M.BF16}[args.storage]
    t0 = time.time()
    # Poisson-disk nodes for the fully scattered set; the hybrid set keeps its
    # jittered-lattice zone, which meets the lattice without a seam (a
    # Poisson-disk zone against the lattice diverges at s = 2)
    poisson = not (args.stratified or args.hybrid)
    ns = nodesets.karman(n_target=args.nodes, hybrid=args.hybrid, poisson=poisson)
    # streaming distance from the finest spacing (refined ring around the
    # cylinder): s = 1 keeps dx <= h everywhere
    dx = units.delta_x(ns.h_min, args.s)
    re = 100.0 * args.s
    tau = units.tau_for_reynolds(0.05, 1.0, dx, re)
    tau_m = 0.5 + (3.0 / 16.0) / (tau - 0.5) if args.trt else tau
    K = args.K
    b = M.build_stencils_for(ns, K, dx, lattice_h=ns.h if args.hybrid else 0.0, reorder=args.reorder)
    perm = b["perm"]
    n_lag = b["n_lagrange"]
    print(f"# built {ns.n} nodes ({n_lag} block centres), K={K}, dx={dx:.4g}, tau={tau:.4f} in "
          f"{time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    cpu_out = None
    if not args.no_cpu_baseline:
        # the oracle on the host, before anything touches the GPU (its
        # all-core leg forks worker processes)
        import copy

        nsp = copy.copy(ns)
        nsp.xy = ns.xy[perm]
        nsp.kind = ns.kind[perm]
        nsp.bc = ns.boundary_values()[perm]
        workers = min(16, os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16")))
        cpu_out = cpu_baseline(nsp, b, tau, workers=workers)
        cpu_out["host_threads_available"] = os.cpu_count()
        print(f"# oracle on the host: {cpu_out['value']:.3f} MNUPS on 1 core, "
              f"{cpu_out.get('all_cores', {}).get('value', float('nan')):.3f} on {workers}", file=sys.stderr,
              flush=True)
    ws_geoms = None
    if not args.no_warm_start:
        # the warm-start media, also before the GPU is touched (worker processes)
        ws_geoms = warmstart_geometries(WS_BENCH[0] + WS_BENCH[1])
    sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=M.POPULATIONS,
                       storage=storage, tau_plus=tau, tau_minus=tau_m, bc=ns.boundary_values()[perm],
                       block=args.block, xcd_remap=args.xcd, scale_exp=12,
                       alternate_sweeps=args.sweeps, cached_weights=args.cached,
                       tile=args.tile, lagrange=b["lagrange"], w_lagrange=b["w_lagrange"],
                       stochastic_rounding=args.sr, weights16=args.weights16,
                       hybrid_launches=args.hybrid_launches)
    n = ns.n
    sim.init_state(np.ones(n), np.zeros((n, 2)))
    per_launch_s = timed_steps(sim, args.steps, args.warmup, torch)
    ms = per_launch_s * 1e3 * args.steps
    _, _, red = sim.macroscopic(dx, want_fields=False)
    red = red.cpu().numpy()
    if red[M._lib.RED_N_BAD] != 0:
        print(f"# warning: {int(red[M._lib.RED_N_BAD])} unstable nodes", file=sys.stderr)
    mnups = n * args.steps / (ms / 1e3) / 1e6
    kp = sim.sizes.k_padded
    bpn_rbf = units.algorithmic_bytes_per_node(M.POPULATIONS, storage, kp, args.weights16)
    bpn_lag = units.block_centre_bytes_per_node(M.POPULATIONS, storage)
    bpn = ((n - n_lag) * bpn_rbf + n_lag * bpn_lag) / n
    achieved = bpn * n / per_launch_s / 1e9
    workload = (f"karman{'-hybrid' if args.hybrid else ''}{'-poisson' if poisson else ''}-n{n}-K{K}-s{args.s:g}"
                + ("" if args.storage == "f32" else f"-{args.storage}") + ("-w16" if args.weights16 else ""))
    kernel = "k_step_pop" + ("_lds" if args.tile else "")
    if args.hybrid and args.tile and args.hybrid_launches == 0:
        kernel = "k_step_pop_hyb"       # both node kinds in one launch per step
    traffic = measured_traffic(kernel, workload)
    out = {
        "metric": METRIC,
        "value": round(mnups, 1),
        "unit": "MNUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32 state+weights, f64 registers",
                  "f16s": f"f16 state (scaled offsets), {'f16' if args.weights16 else 'f32'} weights, f32 registers",
                  "bf16": f"bf16 state, {'f16' if args.weights16 else 'f32'} weights, f32 registers"}[args.storage],
        "data": "synthetic",
        "config": {"workload": "Karman street channel 22Dx4.1D, cylinder D at (2D,2D), " +
                               (f"{n} nodes, hybrid: {n_lag} on a square lattice (biquadratic Lagrange), "
                                f"{n - n_lag} scattered near the cylinder and in its wake "
                                f"({'Poisson-disk, ' if poisson else 'stratified, '}4x denser within "
                                "1D of the cylinder), " if args.hybrid else
                                f"{n} scattered nodes ({'Poisson-disk, ' if poisson else 'stratified, '}"
                                "4x denser within 1D of the cylinder), ") +
                               f"K={K}, s={args.s:g} (Re={re:g}), " + (f"TRT tau+={tau:.4f} tau-={tau_m:.4f}, " if args.trt else f"BGK tau={tau:.4f}, ") + 
                               f"{args.storage} populations",
                   "nodes": n, "block_centres": n_lag, "K": K, "s": args.s, "block": args.block,
                   "xcd_remap": args.xcd,
                   "alternate_sweeps": args.sweeps,
                   "cached_weights": args.cached, "tile": args.tile, "reorder": args.reorder,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kernel, "bytes_per_node": round(bpn, 2),
                     "avg_launch_us": round(per_launch_s * 1e6, 2)},
    }
    del sim
    if not args.no_s_sweep:
        out["s_sweep"] = karman_s_sweep(M, units, np, torch, ns, args, storage, tau, tau_m)
    if not args.no_extra_rows and not args.hybrid:
        # the paper's precision (FP64) on the same set, and the FP32 step on a
        # set five times the memory-side cache
        out["fp64"] = karman_precision_row(M, units, np, torch, ns, b, tau, tau_m, "F64")
        print(f"# f64 row: {out['fp64']['MNUPS']} MNUPS, frac {out['fp64']['frac']}", file=sys.stderr, flush=True)
        out["large_set"] = karman_large_row(M, units, nodesets, np, torch)
        print(f"# large set: {out['large_set']['MNUPS']} MNUPS, frac {out['large_set']['frac']}", file=sys.stderr,
              flush=True)
    if not args.no_steady:
        out["time_to_steady"] = porous_time_to_steady(M, units, nodesets, np, torch)
        out["time_to_steady_inertial"] = porous_time_to_steady(M, units, nodesets, np, torch, s=4.0,
                                                               runs=TTS_RUNS_INERTIAL)
    if ws_geoms is not None:
        geoms, t_geo = ws_geoms
        ws = warmstart_workload(np, torch, WS_BENCH[0], WS_BENCH[1], WS_BENCH[2], geoms=geoms)
        ws["data"]["geometry_s"] = round(t_geo, 1)
        out["warm_start"] = ws
        print(f"# warm start: steps {ws['steps_rest_mean']:.0f} -> {ws['steps_warm_mean']:.0f} "
              f"(x{ws['step_ratio_rest_over_warm']:.3f}), k err max {ws['permeability_rel_err_max']:.2e}",
              file=sys.stderr, flush=True)
    if cpu_out is not None:
        out["cpu_baseline"] = cpu_out
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
