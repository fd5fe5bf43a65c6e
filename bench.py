"""Benchmark of the fused LB-IB time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2|cfg3|cfg1]

Workload (default): the 10 um x 100 um capillary at dx = 50 nm, 2000 x 200
nodes, float32, 18 red cells (352 markers each), 12 adhesive 1 um particles
(6 rigid, 6 soft), receptors on every wall node, Philox bond kinetics; the
whole time step (binning + bonds, membrane and particle forces, fused
collide-stream-spread, interpolation + marker advance) runs each step.

Prints one JSON line: MLUPS (million lattice-node updates per second of the
whole step), the roofline of the dominant kernel (the fused lattice kernel,
timed live with HIP events on its stream) and the FP64 oracle timed on a
bounded sample on the host CPU.
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
    with open(os.path.join(ROOT, "paper_1907_00080_amd", "csrc", "k_lattice.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def make_workload(name: str):
    from workloads import configs
    if name == "cfg2":
        return configs.cfg2_capillary_fp32()
    if name == "cfg3":
        return configs.cfg3_fine_fp32()
    if name == "cfg1":
        w = configs.cfg1_plain_fp64()
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
    return {"value": wl.nodes * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{wl.name}: {n} steps of the full lattice with all bodies (after 1 warm-up "
                      f"step), float64 NumPy, one thread, {dt:.1f} s"}


def traffic_from_profile(bytes_alg: float):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken with the current kernel source; else None."""
    try:
        with open(PROFILE_TRAFFIC) as f:
            rec = json.load(f)
    except Exception:
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--tile", default="64x4")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not part of this "
              "build (see DESIGN.md for how the lattice would be sharded)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1907_00080_amd as pkg

    tile = tuple(int(v) for v in args.tile.split("x"))
    wl = make_workload(args.workload)
    print(f"bench: workload {wl.name} nodes={wl.nodes} markers={wl.n_markers} "
          f"bodies={len(wl.bodies)}", file=sys.stderr, flush=True)
    sim = pkg.Sim(wl, dtype="f32", tile=tile, device="cuda:0", graph_steps=args.graph_steps)
    stream = sim.stream
    sim.step(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    ms_step = ms / args.steps
    mlups = wl.nodes * args.steps / (ms / 1e3) / 1e6
    d = sim.diagnostics()
    print(f"bench: {args.steps} steps in {ms:.1f} ms (wall {wall:.2f} s), {ms_step * 1e3:.2f} us/step, "
          f"{mlups:.0f} MLUPS, nonfinite={d['nonfinite']}", file=sys.stderr, flush=True)
    if d["nonfinite"]:
        raise SystemExit("non-finite state after the benchmark")

    # dominant kernel: fused collide-stream-spread, timed alone on its stream
    k_ms = sim.time_lattice_kernel(50)
    bytes_alg = 72.0 * wl.nodes           # 9 loads + 9 stores of 4 B per node
    achieved = bytes_alg / (k_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(bytes_alg),
            "kernel": "k_lb_fused", "kernel_us": round(k_ms * 1e3, 3),
            "bytes_per_launch": bytes_alg}

    out = {
        "metric": "MLUPS of fused LB-IB step",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "nodes": wl.nodes,
                   "rbc": sum(b.kind == 0 for b in wl.bodies),
                   "particles": sum(b.kind != 0 for b in wl.bodies),
                   "markers": wl.n_markers, "tile": args.tile, "graph_steps": args.graph_steps},
        "roofline": roof,
    }
    if not args.no_cpu:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
