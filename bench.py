"""Benchmark of the fused LB-IB time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload capillary-6667x667|capillary-2000x200|channel-256x64]

Headline workload (default): the fine-mesh capillary of the paper's Sec. 3,
10 um x 100 um at dx = 15 nm, 6667 x 667 nodes (4.45 M), float32, 18 red
cells (1152 markers each), 3 adhesive 1 um particles (rigid, sigma = 0.5, 1,
2), receptors on every wall node, Philox bond kinetics; the whole time step
(bonds, membrane and particle forces, fused collide-stream-spread,
interpolation + marker advance + binning) runs each step.  Its two
population buffers (320 MB) exceed the 256 MB last-level cache, so the
fused lattice kernel streams from HBM.

Prints one JSON line: MLUPS of the whole step over exactly K steps replayed
from captured HIP graphs (and the median of five such windows), the
roofline of the step's dominant kernel (the fused lattice kernel, timed
in-step with HIP events bound to its dispatches), the oracle timed on a
bounded window of the same workload on one host core, and extra objects:
the all-soft variant of the same capillary, the cache-resident 2000 x 200
capillary, a sweep of 64 uneven instances as one autotuned batch against
the same instances run one by one (plain, and graph-captured with tuned
tiles) and against the oracle over all host cores, the gradient window,
and the optional physics of the library (repulsion, MLS transfer,
observables, velocity-wall adhesion boxes).
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
    host launchers, line comments and blank lines left out), which the stored
    counter figures are tied to."""
    with open(os.path.join(ROOT, "paper_1907_00080_amd", "csrc", "k_lattice.hip"), "rb") as f:
        text = f.read()
    cut = text.find(b"// ------------------------------------------------------------------ launchers")
    code = []
    for line in (text if cut < 0 else text[:cut]).split(b"\n"):
        line = line.split(b"//", 1)[0].rstrip()
        if line:
            code.append(line)
    return hashlib.sha256(b"\n".join(code)).hexdigest()[:16]


def make_workload(name: str):
    from workloads import configs
    if name == "capillary-2000x200":
        return configs.capillary_2000x200()
    if name == "capillary-6667x667":
        return configs.capillary_6667x667()
    if name == "capillary-6667x667-soft":
        return configs.capillary_6667x667(soft=True)
    if name == "channel-256x64":
        w = configs.channel_256x64()
        w.dtype = "f32"
        return w
    raise SystemExit(f"unknown workload {name}")


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(name: str, budget_s: float = 20.0, min_steps: int = 3) -> dict:
    """FP64 oracle on one host core: as many steps of the same workload as fit
    the budget (at least `min_steps`), after one untimed step."""
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
    while n < min_steps or time.perf_counter() - t0 < budget_s:
        sim.step(1)
        n += 1
    dt = time.perf_counter() - t0
    if limiter is not None and hasattr(limiter, "unregister"):
        limiter.unregister()
    return {"value": wl.nodes * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "host_cpu": _host_cpu(), "host_threads": os.cpu_count(),
            "sample": f"{wl.name}: a window of {n} steps of the full lattice with all bodies (after "
                      f"1 untimed step), float64 NumPy on one thread, {dt:.1f} s; MLUPS of that "
                      f"window"}


def _oracle_instance_steps(args):
    """Worker of the sweep baseline: oracle steps of one instance on one core
    until the deadline; returns (node updates, seconds)."""
    idx, n_inst, deadline = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle
    from workloads import configs
    wl = configs.sweep_instances(n_inst)[idx]
    sim = oracle.Sim(wl)
    sim.step(1)
    t0 = time.perf_counter()
    n = 0
    while n < 1 or time.time() < deadline:
        sim.step(1)
        n += 1
    return wl.nodes * n, time.perf_counter() - t0


def cpu_baseline_sweep(n_inst: int, budget_s: float = 20.0) -> dict:
    """FP64 oracle on the sweep's instances fanned out over all host cores (one
    process per core, each stepping one instance until the deadline); MLUPS
    = sum of node updates over the pool's wall time."""
    import concurrent.futures
    import multiprocessing
    cores = os.cpu_count() or 1
    nproc = min(cores, n_inst)
    ctx = multiprocessing.get_context("spawn")
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=nproc, mp_context=ctx) as ex:
        # the deadline leaves every worker time to import and set up first
        deadline = time.time() + 10.0 + budget_s
        res = list(ex.map(_oracle_instance_steps, [(i, n_inst, deadline) for i in range(nproc)]))
    wall = time.perf_counter() - t0
    upd = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": upd / busy / 1e6, "unit": "MLUPS", "cores": nproc, "kind": "oracle",
            "host_cpu": _host_cpu(), "host_threads": cores,
            "sample": f"instances 0..{nproc - 1} of the {n_inst}-instance sweep, one per process, "
                      f"float64 NumPy on one thread each, each stepped for about {budget_s:.0f} s "
                      f"(longest {busy:.1f} s, pool wall {wall:.1f} s); MLUPS = node updates of "
                      f"all processes / longest stepping time"}


def traffic_from_profile(workload_name: str, tile=None, hints=None, launch=0, streaming=None):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), if
    it was taken with the current kernel source and (when given) the same tile
    shape, cache hints and population streaming, for the one-workgroup-per-tile
    launch; else None.  The summary holds one configuration per workload and
    optionally further "variants" of it; the cache hints only matter with two
    buffers (in place the kernel uses none)."""
    if launch:
        return None
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except Exception:
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    entries = []
    if workload_name in rec.get("bytes_per_launch", {}):
        entries.append({"tile": rec.get("tiles", {}).get(workload_name),
                        "cache_hints": rec.get("cache_hints", {}).get(workload_name),
                        "streaming": rec.get("streaming", {}).get(workload_name, 0),
                        "bytes_per_launch": rec["bytes_per_launch"][workload_name]})
    entries += [v for v in rec.get("variants", []) if v.get("workload") == workload_name]
    for e in entries:
        st = int(e.get("streaming", 0))
        if tile is not None and e.get("tile") != f"{tile[0]}x{tile[1]}":
            continue
        if streaming is not None and st != int(streaming):
            continue
        if hints is not None and st == 0 and e.get("cache_hints") != int(hints):
            continue
        return e["bytes_per_launch"]
    return None


def tuned_config(pkg, wl, args):
    """Tile shape and step form for one workload: the autotuner's pick (whole
    steps of this workload timed for every tile and step form), or the tile
    given on the command line with the default step form."""
    if args.tile != "auto":
        return (tuple(int(v) for v in args.tile.split("x")), args.step_mode, args.hints, args.launch,
                args.streaming, None)
    from paper_1907_00080_amd import tune
    rec = tune.autotune([wl], dtype="f32", device="cuda:0", steps=200, warmup=20,
                        graph_steps=(args.graph_steps,))
    tile = tuple(rec["tile"])
    launch = int(rec.get("lattice_launch", 0))
    streaming = int(rec.get("streaming", 0))
    print(f"bench: {wl.name} tuned: tile {tile[0]}x{tile[1]}, step mode {rec['step_mode']}, "
          f"cache hints {rec['cache_hints']}, lattice launch {launch}, streaming {streaming} "
          f"({len(rec['candidates'])} + {len(rec.get('launch_candidates', []))} + "
          f"{len(rec.get('streaming_candidates', []))} candidates)", file=sys.stderr, flush=True)
    cands = [{"tile": f"{c['tile'][0]}x{c['tile'][1]}", "step_mode": c["step_mode"],
              "cache_hints": c["cache_hints"], "lattice_launch": int(c.get("lattice_launch", 0)),
              "streaming": int(c.get("streaming", 0)),
              "us_per_step": round(c["ms_per_step"] * 1e3, 2)}
             for c in (list(rec["candidates"]) + list(rec.get("launch_candidates", []))[1:]
                       + list(rec.get("streaming_candidates", []))[1:])]
    return tile, rec["step_mode"], rec["cache_hints"], launch, streaming, cands


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="capillary-6667x667")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of K steps; the first is the reported region, the "
                         "median of all is reported beside it")
    ap.add_argument("--tile", default="auto",
                    help="TXxTY, or auto: tile, step form and cache hints from the autotuner")
    ap.add_argument("--step-mode", type=int, default=None,
                    help="with a fixed --tile: step form (1 three kernels, 2 merged, 3 overlapped)")
    ap.add_argument("--launch", type=int, default=0,
                    help="lattice-kernel launch with a fixed --tile: 0 one workgroup per tile, "
                         "1/2/4/8 persistent workgroups per CU")
    ap.add_argument("--streaming", type=int, default=None,
                    help="population streaming with a fixed --tile: 0 two buffers, 1 in place "
                         "(default: the library's automatic choice)")
    ap.add_argument("--hints", type=int, default=None,
                    help="with a fixed --tile: cache hints of the lattice kernel (0, 1 or 3)")
    ap.add_argument("--side-workload", default="capillary-2000x200",
                    help="workload of the optional-physics objects (repulsion, MLS, observables)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the all-soft and the cache-resident capillaries")
    ap.add_argument("--kernel-steps", type=int, default=200,
                    help="plain-launched steps over which the fused kernel is timed")
    ap.add_argument("--extra-steps", type=int, default=1000)
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
    tile, mode, hints, launch, streaming, cands = tuned_config(pkg, wl, args)
    res = run_workload(pkg, torch, wl, tile, args.steps, args.warmup, args.graph_steps,
                       args.kernel_steps, mode, hints, windows=args.windows, lattice_launch=launch,
                       streaming=streaming)
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
                   "step_mode": res["step_mode"], "cache_hints": res["cache_hints"],
                   "lattice_launch": res["lattice_launch"], "streaming": res["streaming"],
                   "graph_steps": res["graph_steps"], "plain_steps": res["plain_steps"],
                   "graph_prime_steps": res["prime_steps"], "tuned": cands is not None},
        "windows": res["windows"],
        "roofline": roof,
    }
    if cands is not None:
        out["tuning"] = cands
    if not args.no_extra:
        for key, name in (("capillary_6667x667_soft", "capillary-6667x667-soft"),
                          ("capillary_2000x200", "capillary-2000x200")):
            if name == args.workload:
                continue
            xw = make_workload(name)
            xtile, xmode, xhints, xlaunch, xstream, xcands = tuned_config(pkg, xw, args)
            xres = run_workload(pkg, torch, xw, xtile, args.extra_steps, 100, args.graph_steps,
                                args.kernel_steps, xmode, xhints, windows=args.windows,
                                lattice_launch=xlaunch, streaming=xstream)
            xroof = roofline(xres, xw, xtile)
            if 2 * 72.0 * xw.nodes <= 128e6:
                xroof["note"] = ("populations (2 x 36 B per node) stay in the 256 MB last-level "
                                 "cache: a bandwidth figure against the HBM peak, not an HBM-bound "
                                 "roofline; the step is bound by the body kernel's latency")
            out[key] = {"workload": xw.name, "nodes": xw.nodes, "markers": xw.n_markers,
                        "tile": f"{xtile[0]}x{xtile[1]}", "step_mode": xres["step_mode"],
                        "cache_hints": xres["cache_hints"], "lattice_launch": xres["lattice_launch"],
                        "streaming": xres["streaming"],
                        "graph_steps": xres["graph_steps"],
                        "steps": args.extra_steps, "mlups": round(xres["mlups"], 1),
                        "ms_per_step": round(xres["ms_step"], 5), "windows": xres["windows"],
                        "roofline": xroof}
    if not args.no_batch:
        out["batched"] = batched_vs_plain(pkg, torch, args, args.batch_instances, args.batch_steps)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_window(pkg, torch, args.adjoint_steps, 100)
    side = args.side_workload
    if not args.no_repulsion:
        # its own tile: the repulsion reads the marker bins, whose shape follows the tile
        rw = make_workload(side)
        from workloads import configs
        rw.repulsion = configs.REPULSION_COEFF
        rtile = tuned_config(pkg, rw, args)[0]
        out["repulsion"] = repulsion_cost(pkg, torch, side, rtile, 1000, args.graph_steps)
        out["repulsion"]["tile"] = f"{rtile[0]}x{rtile[1]}"
    stile = tuned_config(pkg, make_workload(side), args)[0] if not (args.no_mls and args.no_observables) else None
    if not args.no_mls:
        out["mls"] = mls_cost(pkg, torch, side, stile, 1000, args.graph_steps)
    if not args.no_observables:
        out["observables"] = observables_cost(pkg, torch, side, stile, args.graph_steps)
    if not args.no_couette:
        out["couette_box"] = couette_box_batch(pkg, torch, args.couette_steps)
    if not args.no_cpu:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
        if "batched" in out:
            out["batched"]["cpu_baseline"] = cpu_baseline_sweep(args.batch_instances)
    print(json.dumps(out), flush=True)


def graph_chunk(requested: int, steps: int) -> int:
    """Steps per captured graph for a timed region of `steps` steps: the
    requested chunk, or `steps` itself when that is shorter, rounded down to
    an even number (a graph holds both population-buffer parities); 0 when
    fewer than two steps are timed."""
    g = min(int(requested), int(steps))
    g -= g & 1
    return g if g >= 2 else 0


def run_workload(pkg, torch, wl, tile, steps, warmup, graph_steps, kernel_steps, step_mode=None,
                 cache_hints=None, windows=5, lattice_launch=0, streaming=None):
    """W warm-up steps, then graph capture of both buffer parities (2 chunks,
    untimed), then exactly `steps` steps replayed from the graphs, bracketed by
    HIP events after a device synchronisation; then `windows - 1` more such
    windows (their median is reported beside the first); then the fused
    lattice kernel in-step over `kernel_steps` plain-launched steps."""
    print(f"bench: workload {wl.name} nodes={wl.nodes} markers={wl.n_markers} "
          f"bodies={len(wl.bodies)} tile {tile[0]}x{tile[1]}", file=sys.stderr, flush=True)
    G = graph_chunk(graph_steps, steps)
    sim = pkg.Sim(wl, dtype="f32", tile=tile, device="cuda:0", graph_steps=G,
                  streaming=None if streaming is None else int(streaming))
    if step_mode is not None:
        sim.set_step_mode(int(step_mode))
    if cache_hints is not None:
        sim.set_cache_hints(int(cache_hints))
    sim.set_lattice_launch(int(lattice_launch or 0))
    stream = sim.stream
    sim.step(warmup)
    sim.step(2 * G)                  # captures the graphs of both parities
    times = []
    wall = 0.0
    for w in range(max(1, int(windows))):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(stream)
        sim.step(steps)
        end.record(stream)
        torch.cuda.synchronize()
        if w == 0:
            wall = time.perf_counter() - t0
        times.append(start.elapsed_time(end))
    ms = times[0]
    ms_step = ms / steps
    mlups = wl.nodes * steps / (ms / 1e3) / 1e6
    med = sorted(times)[len(times) // 2]
    d = sim.diagnostics()
    print(f"bench: {steps} steps in {ms:.1f} ms (wall {wall:.2f} s), {ms_step * 1e3:.2f} us/step, "
          f"{mlups:.0f} MLUPS (median of {len(times)} windows {med / steps * 1e3:.2f} us/step), "
          f"graphs of {G}, nonfinite={d['nonfinite']} bin_overflow={d['bin_overflow']}",
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
    hints_used = sim.cache_hints
    launch_used = sim.lattice_launch
    streaming_used = sim.streaming
    sim.close()
    return {"mlups": mlups, "ms_step": ms_step, "kernel_ms": k_ms, "kernel_launches": k_n,
            "step_mode": mode, "cache_hints": hints_used, "lattice_launch": launch_used,
            "streaming": streaming_used,
            "graph_steps": G,
            "plain_steps": steps % G if G else steps, "prime_steps": 2 * G,
            "windows": {"count": len(times), "ms_per_step": [round(t / steps, 5) for t in times],
                        "median_ms_per_step": round(med / steps, 5),
                        "median_mlups": round(wl.nodes * steps / (med / 1e3) / 1e6, 1)}}


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


def batched_vs_plain(pkg, torch, args, n_inst, steps):
    """Sweep of uneven capillary instances (20-100 um long, 200 rows): one
    batch with autotuned tile, step form, cache hints and graph chunk, against
    the same instances run one after another (a) through plain launches (no
    graphs, default tile) and (b) graph-captured with the configuration the
    autotuner picks for a single instance of median length."""
    from workloads import configs
    from paper_1907_00080_amd.tune import autotune
    ws = configs.sweep_instances(n_inst)
    nodes = sum(w.nodes for w in ws)
    print(f"bench: sweep of {len(ws)} instances, {nodes} nodes, "
          f"{sum(w.n_markers for w in ws)} markers; autotuning", file=sys.stderr, flush=True)
    tuned = autotune(ws, "f32", device="cuda:0", steps=100, warmup=20)
    tile = tuple(tuned["tile"])
    b = pkg.Batch(ws, dtype="f32", tile=tile, device="cuda:0", graph_steps=tuned["graph_steps"],
                  streaming=int(tuned.get("streaming", 0)))
    b.set_step_mode(tuned["step_mode"])
    b.set_cache_hints(tuned["cache_hints"])
    b.set_lattice_launch(int(tuned.get("lattice_launch", 0)))
    b.step(2 * max(20, tuned["graph_steps"]))
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
    # (a) plain sequential
    ms_p = 0.0
    for w in ws:
        s = pkg.Sim(w, dtype="f32", tile=(64, 4), device="cuda:0", graph_steps=0)
        s.step(5)
        ms_p += _timed(torch, s, steps)
        s.close()
    # (b) graph-captured sequential, tuned on the instance of median length
    order = sorted(range(len(ws)), key=lambda i: ws[i].nodes)
    rep = ws[order[len(order) // 2]]
    one = autotune([rep], "f32", device="cuda:0", steps=100, warmup=20, graph_steps=(100,))
    ms_g = 0.0
    for w in ws:
        s = pkg.Sim(w, dtype="f32", tile=tuple(one["tile"]), device="cuda:0", graph_steps=100,
                    streaming=int(one.get("streaming", 0)))
        s.set_step_mode(one["step_mode"])
        s.set_cache_hints(one["cache_hints"])
        s.set_lattice_launch(int(one.get("lattice_launch", 0)))
        s.step(200)
        ms_g += _timed(torch, s, steps)
        s.close()
    mb = nodes * steps / (ms_b * 1e-3) / 1e6
    mp = nodes * steps / (ms_p * 1e-3) / 1e6
    mg = nodes * steps / (ms_g * 1e-3) / 1e6
    print(f"bench: batched {mb:.0f} MLUPS (tile {tile[0]}x{tile[1]}, graphs of "
          f"{tuned['graph_steps']}, step mode {tuned['step_mode']}, hints {tuned['cache_hints']}), "
          f"sequential plain {mp:.0f} MLUPS, sequential graph-captured tuned {mg:.0f} MLUPS; "
          f"batched lattice kernel {k_ms * 1e3:.1f} us "
          f"({72.0 * nodes / (k_ms / 1e3) / 1e9:.0f} GB/s of algorithmic traffic)",
          file=sys.stderr, flush=True)
    return {"workload": f"sweep-{len(ws)}-instances", "instances": len(ws), "nodes": nodes,
            "steps": steps, "batched_mlups": round(mb, 1), "plain_mlups": round(mp, 1),
            "speedup": round(mb / mp, 3),
            "sequential_graph_tuned_mlups": round(mg, 1), "speedup_vs_graph_tuned": round(mb / mg, 3),
            "sequential_graph_tuned_config": {"tile": f"{one['tile'][0]}x{one['tile'][1]}",
                                              "step_mode": one["step_mode"],
                                              "cache_hints": one["cache_hints"],
                                              "lattice_launch": int(one.get("lattice_launch", 0)),
                                              "tuned_on": rep.name},
            "tile": f"{tile[0]}x{tile[1]}", "cache_hints": tuned["cache_hints"],
            "lattice_kernel": {"kernel_us": round(k_ms * 1e3, 3), "launches": k_n,
                               "bytes_per_launch": 72.0 * nodes,
                               "achieved": round(72.0 * nodes / (k_ms / 1e3) / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(72.0 * nodes / (k_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
            "graph_steps": tuned["graph_steps"], "step_mode": tuned["step_mode"],
            "lattice_launch": int(tuned.get("lattice_launch", 0)),
            "streaming": int(tuned.get("streaming", 0)),
            "streaming_candidates": [{"streaming": int(c["streaming"]), "mlups": round(c["mlups"], 1),
                                      "us_per_step": round(c["ms_per_step"] * 1e3, 2)}
                                     for c in tuned.get("streaming_candidates", [])],
            "candidates": [{"tile": f"{c['tile'][0]}x{c['tile'][1]}", "graph_steps": c["graph_steps"],
                            "step_mode": c["step_mode"], "cache_hints": c["cache_hints"],
                            "mlups": round(c["mlups"], 1)}
                           for c in tuned["candidates"]],
            # the lattice kernel's launch form at the pick: 0 one workgroup per
            # tile, w > 0 a persistent grid of w workgroups per CU
            "launch_candidates": [{"lattice_launch": int(c["lattice_launch"]),
                                   "mlups": round(c["mlups"], 1),
                                   "us_per_step": round(c["ms_per_step"] * 1e3, 2)}
                                  for c in tuned.get("launch_candidates", [])]}


FD_PARAMS = ((1, 0, "ks_particle"), (1, 1, "kb_particle"), (1, 2, "sigma_particle"),
             (0, 0, "ks_rbc"))


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
        # median of three repetitions of each (wall clock around whole calls)
        t_fwds, t_adjs = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            t_fwds.append(time.perf_counter() - t0)
            sim.set_state(state)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            J, nb = win.forward()
            g = win.backward(1.0)
            torch.cuda.synchronize()
            t_adjs.append(time.perf_counter() - t0)
            sim.set_state(state)
        t_fwd, t_adj = sorted(t_fwds)[1], sorted(t_adjs)[1]
        res[dtype] = dict(J=J, g=g, t_fwd=t_fwd, t_adj=t_adj, bonds=nb)
        if dtype == "f64":
            # central differences of the float64 forward (h = 1e-4 relative):
            # the reference for both adjoints
            fds = {}
            for (b, q, name) in FD_PARAMS:
                h = 1e-4 * P0[b, q]
                Js = []
                for sgn in (1, -1):
                    P = P0.copy()
                    P[b, q] += sgn * h
                    sim.set_state(state)
                    params(P, sim)
                    Js.append(win.forward()[0])
                fds[name] = (Js[0] - Js[1]) / (2 * h)
        sim.close()
    for dtype in ("f32", "f64"):
        g = res[dtype]["g"]
        res[dtype]["fd_rel_err"] = {name: abs(g[b, q] - fds[name]) / abs(fds[name])
                                    for b, q, name in FD_PARAMS}
    r32, r64 = res["f32"], res["f64"]
    ratio = r32["t_adj"] / r32["t_fwd"]
    g32, g64 = r32["g"], r64["g"]
    sel = [(1, 0), (1, 1), (1, 2), (0, 0)]
    f32_vs_f64 = max(abs(g32[b, q] - g64[b, q]) / abs(g64[b, q]) for b, q in sel)
    print(f"bench: adjoint/forward {ratio:.2f} (fp32: forward {1e3 * r32['t_fwd']:.1f} ms, "
          f"adjoint {1e3 * r32['t_adj']:.1f} ms), fp32 adjoint vs FD of the fp64 forward "
          f"{r32['fd_rel_err']}", file=sys.stderr, flush=True)
    return {"workload": wl.name, "steps": steps, "ckpt_every": ckpt, "dtype": "f32 forward, f64 adjoint",
            "adjoint_over_forward": round(ratio, 3),
            "forward_ms": round(1e3 * r32["t_fwd"], 2), "adjoint_ms": round(1e3 * r32["t_adj"], 2),
            "timing": "median of 3 wall-clock repetitions of each",
            "J": r32["J"], "bonds": r32["bonds"],
            "grad_fp32": {"ks_particle": g32[1, 0], "kb_particle": g32[1, 1],
                          "sigma_particle": g32[1, 2], "ks_rbc": g32[0, 0]},
            "fp64_adjoint_vs_fp64_fd_rel_err": {k: float(f"{v:.3e}") for k, v in r64["fd_rel_err"].items()},
            "fp32_adjoint_vs_fp64_fd_rel_err": {k: float(f"{v:.3e}") for k, v in r32["fd_rel_err"].items()},
            "fp32_vs_fp64_gradient_rel_diff": float(f"{f32_vs_f64:.3e}"),
            "fp64_adjoint_over_forward": round(r64["t_adj"] / r64["t_fwd"], 3)}


def roofline(res, wl, tile=None):
    bytes_alg = 72.0 * wl.nodes           # 9 loads + 9 stores of 4 B per node
    achieved = bytes_alg / (res["kernel_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(wl.name, tile, res.get("cache_hints"),
                                            res.get("lattice_launch", 0), res.get("streaming")),
            # in place, the step alternates two passes of the kernel (the
            # neighbour pass and the node-local pass): their mean
            "kernel": ("k_lb_persistent" if res.get("lattice_launch") else
                       "k_lb_fused (in place, both passes)" if res.get("streaming") else "k_lb_fused"),
            "kernel_us": round(res["kernel_ms"] * 1e3, 3),
            "launches": res["kernel_launches"], "bytes_per_launch": bytes_alg}


if __name__ == "__main__":
    main()
