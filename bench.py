"""Benchmark of the fused LB-IB time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload capillary-2000x200|capillary-6667x667|channel-256x64]

Workload (default): the 10 um x 100 um capillary at dx = 50 nm, 2000 x 200
nodes, float32, 18 red cells (352 markers each), 12 adhesive 1 um particles
(6 rigid, 6 soft), receptors on every wall node, Philox bond kinetics; the
whole time step (binning + bonds, membrane and particle forces, fused
collide-stream-spread, interpolation + marker advance) runs each step.

Prints one JSON line: MLUPS (million lattice-node updates per second of the
whole step, graph-captured chunks of steps), the roofline of the dominant
kernel (the fused lattice kernel, timed in-step with HIP events bound to its
dispatches over plain-launched steps of the same run), the same figures for
the HBM-bound 6667 x 667 capillary, a sweep of 64 uneven instances run as one
autotuned batch against the same instances run one by one, and the FP64
oracle timed on a bounded sample on the host CPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "lb_fused_traffic.json")


def kernel_source_hash() -> str:
    """Hash of the fused kernel's device code (the lattice source up to its
    host launchers), which the stored counter figures are tied to."""
    with open(os.path.join(ROOT, "paper_1907_00080_amd", "csrc", "k_lattice.hip"), "rb") as f:
        text = f.read()
    cut = text.find(b"// ------------------------------------------------------------------ launchers")
    return hashlib.sha256(text if cut < 0 else text[:cut]).hexdigest()[:16]


def make_workload(name: str):
    from workloads import configs
    if name == "capillary-2000x200":
        return configs.capillary_2000x200()
    if name == "capillary-6667x667":
        return configs.capillary_6667x667()
    if name == "channel-256x64":
        w = configs.channel_256x64()
        w.dtype = "f32"
        return w
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(name: str, budget_s: float = 15.0) -> dict:
    """FP64 oracle on the host: as many steps of the same workload as fit the budget."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        limiter = None
    wl = make_workload(name)
    sim = oracle.Sim(wl)
    sim.step(1)                     # first step pays one-off costs
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s:
        sim.step(1)
        n += 1
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": wl.nodes * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_threads": os.cpu_count(),
            "sample": f"{wl.name}: {n} steps of the full lattice with all bodies (after 1 warm-up "
                      f"step), float64 NumPy, one thread, {dt:.1f} s"}


def traffic_from_profile(workload_name: str, tile=None):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), if
    it was taken with the current kernel source and (when given) the same tile
    shape; else None."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except Exception:
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if tile is not None and rec.get("tiles", {}).get(workload_name) != f"{tile[0]}x{tile[1]}":
        return None
    return rec.get("bytes_per_launch", {}).get(workload_name)


def tuned_config(pkg, wl, args):
    """Tile shape and step form for one workload: the autotuner's pick (whole
    steps of this workload timed for every tile and step form), or the tile
    given on the command line with the default step form."""
    if args.tile != "auto":
        return tuple(int(v) for v in args.tile.split("x")), None, None, None
    from paper_1907_00080_amd import tune
    rec = tune.autotune([wl], dtype="f32", device="cuda:0", steps=200, warmup=20,
                        graph_steps=(args.graph_steps,))
    tile = tuple(rec["tile"])
    print(f"bench: {wl.name} tuned: tile {tile[0]}x{tile[1]}, step mode {rec['step_mode']}, "
          f"cache hints {rec['cache_hints']} ({len(rec['candidates'])} candidates)",
          file=sys.stderr, flush=True)
    cands = [{"tile": f"{c['tile'][0]}x{c['tile'][1]}", "step_mode": c["step_mode"],
              "cache_hints": c["cache_hints"], "us_per_step": round(c["ms_per_step"] * 1e3, 2)}
             for c in rec["candidates"]]
    return tile, rec["step_mode"], rec["cache_hints"], cands


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="capillary-2000x200")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--tile", default="auto",
                    help="TXxTY, or auto: tile and step form from the autotuner, per workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 6667 x 667 capillary")
    ap.add_argument("--kernel-steps", type=int, default=200,
                    help="plain-launched steps over which the fused kernel is timed")
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain sweep")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient window")
    ap.add_argument("--no-couette", action="store_true",
                    help="skip the adhesion boxes with velocity walls")
    ap.add_argument("--couette-steps", type=int, default=2000)
    ap.add_argument("--no-repulsion", action="store_true",
                    help="skip the step with the vertex repulsion switched on")
    ap.add_argument("--no-mls", action="store_true",
                    help="skip the step with the moving-least-squares transfer")
    ap.add_argument("--no-observables", action="store_true",
                    help="skip the on-device observations")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--batch-instances", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 320 MiB x 10 (for counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not supported "
              "(a single capillary would be sharded in slabs along x with a population halo "
              "exchange, a sweep by instances)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        # reference for the HBM byte counters: each copy reads and writes 320 MiB
        a = torch.ones(80 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4,
                          "copies": 10}), flush=True)
        return
    import paper_1907_00080_amd as pkg

    wl = make_workload(args.workload)
    tile, mode, hints, cands = tuned_config(pkg, wl, args)
    res = run_workload(pkg, torch, wl, tile, args.steps, args.warmup, args.graph_steps,
                       args.kernel_steps, mode, hints)
    roof = roofline(res, wl, tile)

    out = {
        "metric": "MLUPS of fused LB-IB step; batched vs plain MLUPS; adjoint/forward time",
        "value": round(res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nodes": wl.nodes,
                   "rbc": sum(b.kind == 0 for b in wl.bodies),
                   "particles": sum(b.kind != 0 for b in wl.bodies),
                   "markers": wl.n_markers, "tile": f"{tile[0]}x{tile[1]}",
                   "step_mode": res["step_mode"], "graph_steps": args.graph_steps,
                   "tuned": cands is not None},
        "roofline": roof,
    }
    if cands is not None:
        out["tuning"] = cands
    if not args.no_large and args.workload != "capillary-6667x667":
        # the HBM-bound case: 10 um x 100 um capillary at dx = 15 nm
        lw = make_workload("capillary-6667x667")
        ltile, lmode, lhints, lcands = tuned_config(pkg, lw, args)
        lres = run_workload(pkg, torch, lw, ltile, args.large_steps, 20, args.graph_steps,
                            args.large_steps, lmode, lhints)
        out["large_lattice"] = {"workload": lw.name, "nodes": lw.nodes, "markers": lw.n_markers,
                                "tile": f"{ltile[0]}x{ltile[1]}", "step_mode": lres["step_mode"],
                                "mlups": round(lres["mlups"], 1),
                                "ms_per_step": round(lres["ms_step"], 5),
                                "roofline": roofline(lres, lw, ltile)}
    if not args.no_batch:
        out["batched"] = batched_vs_plain(pkg, torch, args.batch_instances, args.batch_steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_window(pkg, torch, args.adjoint_steps, 100)
    if not args.no_repulsion:
        # its own tile: the repulsion reads the marker bins, whose shape follows the tile
        rw = make_workload(args.workload)
        from workloads import configs
        rw.repulsion = configs.REPULSION_COEFF
        rtile = tuned_config(pkg, rw, args)[0]
        out["repulsion"] = repulsion_cost(pkg, torch, args.workload, rtile, 1000, args.graph_steps)
        out["repulsion"]["tile"] = f"{rtile[0]}x{rtile[1]}"
    if not args.no_mls:
        out["mls"] = mls_cost(pkg, torch, args.workload, tile, 1000, args.graph_steps)
    if not args.no_observables:
        out["observables"] = observables_cost(pkg, torch, args.workload, tile, args.graph_steps)
    if not args.no_couette:
        out["couette_box"] = couette_box_batch(pkg, torch, args.couette_steps)
    if not args.no_cpu:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


def run_workload(pkg, torch, wl, tile, steps, warmup, graph_steps, kernel_steps, step_mode=None,
                 cache_hints=None):
    """Time `steps` whole steps (graph-captured chunks), then measure the fused
    lattice kernel in-step over `kernel_steps` plain-launched steps."""
    print(f"bench: workload {wl.name} nodes={wl.nodes} markers={wl.n_markers} "
          f"bodies={len(wl.bodies)} tile {tile[0]}x{tile[1]}", file=sys.stderr, flush=True)
    sim = pkg.Sim(wl, dtype="f32", tile=tile, device="cuda:0", graph_steps=graph_steps)
    if step_mode is not None:
        sim.set_step_mode(int(step_mode))
    if cache_hints is not None:
        sim.set_cache_hints(int(cache_hints))
    stream = sim.stream
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    ms_step = ms / steps
    mlups = wl.nodes * steps / (ms / 1e3) / 1e6
    d = sim.diagnostics()
    print(f"bench: {steps} steps in {ms:.1f} ms (wall {wall:.2f} s), {ms_step * 1e3:.2f} us/step, "
          f"{mlups:.0f} MLUPS, nonfinite={d['nonfinite']} bin_overflow={d['bin_overflow']}",
          file=sys.stderr, flush=True)
    if d["nonfinite"] or d["bin_overflow"] or d["sync_timeouts"]:
        raise SystemExit("invalid state after the benchmark")
    # dominant kernel: fused collide-stream-spread, bracketed by HIP events on
    # its own stream during plain-launched steps of the same run
    sim.set_kernel_timing(True)
    sim.step(kernel_steps)
    k_ms, k_n = sim.kernel_timing()
    sim.set_kernel_timing(False)
    print(f"bench: fused lattice kernel {k_ms * 1e3:.2f} us over {k_n} in-step launches",
          file=sys.stderr, flush=True)
    mode = sim.step_mode
    sim.close()
    return {"mlups": mlups, "ms_step": ms_step, "kernel_ms": k_ms, "kernel_launches": k_n,
            "step_mode": mode}


def repulsion_cost(pkg, torch, name, tile, steps, graph_steps):
    """The same workload with the vertex repulsion (Eq. repFor, the paper's
    coefficient, cutoff 2) switched on, which runs the three-kernel step form
    plus the repulsion kernel; against the same form without it and against
    the default (merged) form without it."""
    from workloads import configs
    res = {}
    for key, coeff, mode in (("on", configs.REPULSION_COEFF, 0), ("off_three_kernel", 0.0, 1),
                             ("off_default", 0.0, 0)):
        wl = make_workload(name)
        wl.repulsion = coeff
        sim = pkg.Sim(wl, dtype="f32", tile=tile, device="cuda:0", graph_steps=graph_steps)
        sim.set_step_mode(mode)
        sim.step(200)
        ms = _timed(torch, sim, steps) / steps
        d = sim.diagnostics()
        if d["nonfinite"] or d["bin_overflow"] or d["sync_timeouts"]:
            raise SystemExit("invalid state after the repulsion benchmark")
        res[key] = {"ms_per_step": round(ms, 5), "mlups": round(wl.nodes / (ms * 1e-3) / 1e6, 1),
                    "step_mode": sim.step_mode}
        sim.close()
    res["workload"] = name + " with vertex repulsion"
    res["repulsion_us_per_step"] = round(1e3 * (res["on"]["ms_per_step"]
                                               - res["off_three_kernel"]["ms_per_step"]), 2)
    print(f"bench: repulsion on {res['on']['ms_per_step'] * 1e3:.2f} us/step, three kernels "
          f"without {res['off_three_kernel']['ms_per_step'] * 1e3:.2f}, default form "
          f"{res['off_default']['ms_per_step'] * 1e3:.2f}", file=sys.stderr, flush=True)
    return res


def mls_cost(pkg, torch, name, tile, steps, graph_steps):
    """The same workload with the general moving-least-squares transfer
    (linear basis, cubic-spline and Gaussian weights of support half-width
    1.3, the paper's 2.6 dx square) in place of the Roma kernel, default step
    form, against the Roma kernel."""
    res = {}
    for key, transfer, weight in (("roma_kernel", "roma", "cubic"), ("mls_cubic", "mls", "cubic"),
                                  ("mls_gauss", "mls", "gauss")):
        wl = make_workload(name)
        wl.transfer, wl.mls_weight, wl.mls_support = transfer, weight, 1.3
        sim = pkg.Sim(wl, dtype="f32", tile=tile, device="cuda:0", graph_steps=graph_steps)
        sim.step(200)
        ms = _timed(torch, sim, steps) / steps
        d = sim.diagnostics()
        if d["nonfinite"] or d["bin_overflow"] or d["sync_timeouts"]:
            raise SystemExit("invalid state after the MLS benchmark")
        res[key] = {"ms_per_step": round(ms, 5), "mlups": round(wl.nodes / (ms * 1e-3) / 1e6, 1),
                    "step_mode": sim.step_mode}
        sim.close()
    res["workload"] = name + " with the MLS transfer"
    print(f"bench: transfer Roma kernel {res['roma_kernel']['ms_per_step'] * 1e3:.2f} us/step, "
          f"MLS cubic {res['mls_cubic']['ms_per_step'] * 1e3:.2f}, MLS Gaussian "
          f"{res['mls_gauss']['ms_per_step'] * 1e3:.2f}", file=sys.stderr, flush=True)
    return res


def observables_cost(pkg, torch, name, tile, graph_steps, every=100, n_obs=20):
    """On-device observations of the workload every `every` steps: the cost
    of one observation (HIP events around it) and the resulting per-region
    counts of the particles at the end."""
    from workloads import configs
    wl = make_workload(name)
    sim = pkg.Sim(wl, dtype="f32", tile=tile, device="cuda:0", graph_steps=graph_steps)
    sim.step(200)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    ms = 0.0
    for _ in range(n_obs):
        start.record(sim.stream)
        sim.observe()
        end.record(sim.stream)
        sim.step(every)
        end.synchronize()
        ms += start.elapsed_time(end)
    recs = sim.observations()
    sim.close()
    parts = [r for r, b in zip(recs, wl.bodies) if b.kind != configs.RBC_KINEMATIC]
    regions = {"cell_free_layer": 0, "intermediate": 0, "bulk": 0}
    names = {0: "cell_free_layer", 1: "intermediate", 2: "bulk"}
    for r in parts:
        regions[names[r["region"]]] += 1
    res = {"workload": name, "bodies": len(recs), "every_steps": every, "observations": n_obs,
           "us_per_observation": round(1e3 * ms / n_obs, 2),
           "particles_by_region": regions,
           "particles_with_bonds": sum(1 for r in parts if r["n_bonds"] > 0),
           "max_r_max_over_H": round(max((r["r_max"] for r in parts), default=0.0) / wl.ny, 6)}
    print(f"bench: observation of {len(recs)} bodies {res['us_per_observation']} us", file=sys.stderr,
          flush=True)
    return res


def couette_box_batch(pkg, torch, steps):
    """The paper's adhesion workload: 600 x 200 boxes at dx = 15 nm between
    Zou-He velocity walls (moving top wall), one 1 um particle each, rigid and
    soft with sigma = 0.5, 1, 2: six instances advanced as one batch.  Reports
    the batch's MLUPS and, per instance, the bonds held and the particle's
    rolling velocity over the timed steps relative to the top wall speed."""
    from workloads import configs
    ws = [configs.couette_box(kind=k, sigma_phys=s)
          for k in (configs.PARTICLE_RIGID, configs.PARTICLE_SOFT) for s in (0.5, 1.0, 2.0)]
    for i, w in enumerate(ws):
        w.instance = i
    nodes = sum(w.nodes for w in ws)
    b = pkg.Batch(ws, dtype="f32", graph_steps=100)
    b.step(200)
    b.observe()
    ms = _timed(torch, b, steps)
    b.observe()
    recs = b.observations()
    d = b.diagnostics()
    b.close()
    if d["nonfinite"] or d["bin_overflow"] or d["sync_timeouts"]:
        raise SystemExit("invalid state after the adhesion boxes")
    inst = [{"instance": w.name, "bonds": r["n_bonds"], "bonds_at_start": r["n_bonds0"],
             "u_roll_over_u_top": round(r["u_x"] / w.u_wall[1], 4)} for w, r in zip(ws, recs)]
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    print(f"bench: adhesion boxes (6 x 600x200, velocity walls) {mlups:.0f} MLUPS", file=sys.stderr,
          flush=True)
    return {"workload": "couette-box-600x200 x6 (rigid, soft; sigma 0.5, 1, 2)", "nodes": nodes,
            "steps": steps, "ms_per_step": round(ms / steps, 5), "mlups": round(mlups, 1),
            "instances": inst}


def _timed(torch, ctx, steps):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    ctx.step(steps)
    end.record(ctx.stream)
    end.synchronize()
    return start.elapsed_time(end)


def batched_vs_plain(pkg, torch, n_inst, steps):
    """Sweep of uneven capillary instances (20-100 um long, 200 rows): one
    batch with autotuned tiles and graph chunks, against the same instances
    run one after another through plain launches (no graphs, default tile)."""
    from workloads import configs
    from paper_1907_00080_amd.tune import autotune
    ws = configs.sweep_instances(n_inst)
    nodes = sum(w.nodes for w in ws)
    print(f"bench: sweep of {len(ws)} instances, {nodes} nodes, "
          f"{sum(w.n_markers for w in ws)} markers; autotuning", file=sys.stderr, flush=True)
    tuned = autotune(ws, "f32", device="cuda:0", steps=100, warmup=20)
    tile = tuple(tuned["tile"])
    b = pkg.Batch(ws, dtype="f32", tile=tile, device="cuda:0", graph_steps=tuned["graph_steps"])
    b.set_step_mode(tuned["step_mode"])
    b.step(max(20, tuned["graph_steps"]))
    ms_b = _timed(torch, b, steps)
    # the fused lattice kernel of the batch (one launch for all instances):
    # HIP events bound to its dispatches over plain-launched steps
    b.set_kernel_timing(True)
    b.step(50)
    k_ms, k_n = b.kernel_timing()
    b.set_kernel_timing(False)
    d = b.diagnostics()
    b.close()
    if d["nonfinite"] or d["bin_overflow"] or d["sync_timeouts"]:
        raise SystemExit("invalid batch state after the benchmark")
    ms_p = 0.0
    for w in ws:
        s = pkg.Sim(w, dtype="f32", tile=(64, 4), device="cuda:0", graph_steps=0)
        s.step(5)
        ms_p += _timed(torch, s, steps)
        s.close()
    mb = nodes * steps / (ms_b * 1e-3) / 1e6
    mp = nodes * steps / (ms_p * 1e-3) / 1e6
    print(f"bench: batched {mb:.0f} MLUPS (tile {tile[0]}x{tile[1]}, graphs of "
          f"{tuned['graph_steps']}, step mode {tuned['step_mode']}), plain sequential {mp:.0f} MLUPS; "
          f"batched lattice kernel {k_ms * 1e3:.1f} us "
          f"({72.0 * nodes / (k_ms / 1e3) / 1e9:.0f} GB/s of algorithmic traffic)",
          file=sys.stderr, flush=True)
    return {"workload": f"sweep-{len(ws)}-instances", "instances": len(ws), "nodes": nodes,
            "steps": steps, "batched_mlups": round(mb, 1), "plain_mlups": round(mp, 1),
            "speedup": round(mb / mp, 3), "tile": f"{tile[0]}x{tile[1]}",
            "lattice_kernel": {"kernel_us": round(k_ms * 1e3, 3), "launches": k_n,
                               "bytes_per_launch": 72.0 * nodes,
                               "achieved": round(72.0 * nodes / (k_ms / 1e3) / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(72.0 * nodes / (k_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
            "graph_steps": tuned["graph_steps"], "step_mode": tuned["step_mode"],
            "candidates": [{"tile": f"{c['tile'][0]}x{c['tile'][1]}", "graph_steps": c["graph_steps"],
                            "step_mode": c["step_mode"], "mlups": round(c["mlups"], 1)}
                           for c in tuned["candidates"]]}


def adjoint_window(pkg, torch, steps, ckpt):
    """Gradient window on the 256 x 64 channel (red cell + soft adhesive
    particle, bonds frozen after the first step): wall time of the adjoint
    (forward window with checkpoints + checkpointed reverse sweep) over the
    wall time of the same steps run forward only; gradient accuracy of the
    float64 adjoint against float64 central differences (h = 1e-4 relative)
    of the GPU forward, and the float32-forward gradient against it."""
    from workloads import configs
    from paper_1907_00080_amd.adjoint import AdjointWindow
    wl = configs.adjoint_channel()
    print(f"bench: gradient window {wl.name}, {steps} steps, checkpoints every {ckpt}",
          file=sys.stderr, flush=True)

    def params(P, sim):
        for b in range(P.shape[0]):
            sim.set_body_params(b, *P[b])

    import numpy as np
    P0 = np.array([[b.ks, b.kb, b.sigma] for b in wl.bodies])
    res = {}
    for dtype in ("f32", "f64"):
        sim = pkg.Sim(wl, dtype=dtype, device="cuda:0", graph_steps=100)
        sim.step(1)
        state = sim.get_state()
        win = AdjointWindow(sim, steps, ckpt)
        sim.step(steps)                       # warm-up: graphs of the forward
        sim.set_state(state)
        win.forward()
        win.backward(1.0)                     # warm-up: graphs of the segments
        sim.set_state(state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        sim.set_state(state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, nb = win.forward()
        g = win.backward(1.0)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        res[dtype] = dict(J=J, g=g, t_fwd=t_fwd, t_adj=t_adj, bonds=nb)
        if dtype == "f64":
            errs = {}
            for (b, q, name) in ((1, 0, "ks_particle"), (1, 2, "sigma_particle"), (0, 0, "ks_rbc")):
                h = 1e-4 * P0[b, q]
                Js = []
                for sgn in (1, -1):
                    P = P0.copy()
                    P[b, q] += sgn * h
                    sim.set_state(state)
                    params(P, sim)
                    Js.append(win.forward()[0])
                fd = (Js[0] - Js[1]) / (2 * h)
                errs[name] = abs(g[b, q] - fd) / abs(fd)
            res[dtype]["fd_rel_err"] = errs
        sim.close()
    r32, r64 = res["f32"], res["f64"]
    ratio = r32["t_adj"] / r32["t_fwd"]
    g32, g64 = r32["g"], r64["g"]
    sel = [(1, 0), (1, 1), (1, 2), (0, 0)]
    f32_vs_f64 = max(abs(g32[b, q] - g64[b, q]) / abs(g64[b, q]) for b, q in sel)
    print(f"bench: adjoint/forward {ratio:.2f} (fp32: forward {1e3 * r32['t_fwd']:.1f} ms, "
          f"adjoint {1e3 * r32['t_adj']:.1f} ms), fp64 FD rel err {r64['fd_rel_err']}",
          file=sys.stderr, flush=True)
    return {"workload": wl.name, "steps": steps, "ckpt_every": ckpt, "dtype": "f32 forward, f64 adjoint",
            "adjoint_over_forward": round(ratio, 3),
            "forward_ms": round(1e3 * r32["t_fwd"], 2), "adjoint_ms": round(1e3 * r32["t_adj"], 2),
            "J": r32["J"], "bonds": r32["bonds"],
            "grad_fp32": {"ks_particle": g32[1, 0], "kb_particle": g32[1, 1],
                          "sigma_particle": g32[1, 2], "ks_rbc": g32[0, 0]},
            "fp64_adjoint_vs_fp64_fd_rel_err": {k: float(f"{v:.3e}") for k, v in r64["fd_rel_err"].items()},
            "fp32_vs_fp64_gradient_rel_diff": float(f"{f32_vs_f64:.3e}"),
            "fp64_adjoint_over_forward": round(r64["t_adj"] / r64["t_fwd"], 3)}


def roofline(res, wl, tile=None):
    bytes_alg = 72.0 * wl.nodes           # 9 loads + 9 stores of 4 B per node
    achieved = bytes_alg / (res["kernel_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(wl.name, tile),
            "kernel": "k_lb_fused", "kernel_us": round(res["kernel_ms"] * 1e3, 3),
            "launches": res["kernel_launches"], "bytes_per_launch": bytes_alg}


if __name__ == "__main__":
    main()
