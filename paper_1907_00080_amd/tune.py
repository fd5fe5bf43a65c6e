"""Autotuner for batched sweeps: tile shape, step form, cache hints, graph chunk,
lattice-kernel launch form and population streaming (host logic).

A batch advances many uneven capillary instances together (one launch per
kernel per step for all of them).  Which tile shape of the fused lattice
kernel, which step form (three kernels, merged marker advance, overlapped
lattice tiles) and which number of steps per captured HIP graph run fastest
depends on the instance mix and the device, and so do the cache hints of the
lattice kernel's population accesses (plain, non-temporal loads, non-temporal
loads and stores), so `autotune` times whole steps of the actual batch for
every candidate and keeps the fastest.  Results are cached in a JSON file
keyed by the batch signature (lattice shapes, wall mode, transfer, repulsion,
body and marker counts, dtype) and the device name, so a sweep pays for
tuning once.

Nothing here computes a step of the method; every step runs in the library.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile
from typing import Callable, Iterable, Optional, Sequence, Tuple

TILES: Tuple[Tuple[int, int], ...] = ((64, 4), (128, 2), (32, 8), (256, 1))
GRAPH_STEPS: Tuple[int, ...] = (10, 100)
STEP_MODES: Tuple[int, ...] = (1, 2, 3)   # three kernels, merged advance, overlapped tiles
CACHE_HINTS: Tuple[int, ...] = (0, 1, 3)   # plain, non-temporal loads, non-temporal loads + stores
# lattice-kernel launch: one workgroup per tile (0) or a persistent grid of
# that many workgroups per CU; timed for the best of the other choices
LATTICE_LAUNCHES: Tuple[int, ...] = (0, 1, 2, 4, 8)
# population streaming: two buffers (0) or one buffer in place (1); timed
# last, at the pick of the other stages (the launch form applies to 0 only)
STREAMINGS: Tuple[int, ...] = (0, 1)


def signature(workloads: Sequence, dtype: str) -> str:
    """Stable key of a batch: dtype plus, per instance, lattice shape, wall
    mode, lattice <-> marker transfer (and MLS weight), whether the vertex
    repulsion is on, body count and marker count: everything that changes
    which kernel variants and step forms run."""
    h = hashlib.sha256()
    h.update(str(dtype).encode())
    for w in workloads:
        walls = getattr(w, "walls", "bounce-back")
        transfer = getattr(w, "transfer", "roma")
        weight = getattr(w, "mls_weight", "cubic") if transfer == "mls" else "-"
        rep = 1 if float(getattr(w, "repulsion", 0.0)) > 0.0 else 0
        h.update(f"{int(w.nx)}x{int(w.ny)}:{int(w.periodic_y)}:{walls}:{transfer}:{weight}:"
                 f"{rep}:{len(w.bodies)}:{int(w.n_markers)};".encode())
    return h.hexdigest()[:24]


def load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def store_cache(path: str, key: str, record: dict) -> None:
    """Add one record; the file is replaced atomically."""
    data = load_cache(path)
    data[key] = record
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(results: Iterable[dict]) -> dict:
    """Fastest candidate; ties go to the earlier one (candidate order)."""
    best = None
    for r in results:
        if best is None or r["ms_per_step"] < best["ms_per_step"]:
            best = r
    if best is None:
        raise ValueError("no tuning results")
    return best


def _time_steps(batch, steps: int) -> float:
    """Milliseconds for `steps` steps of `batch`, HIP events on its stream."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(batch.stream)
    batch.step(steps)
    end.record(batch.stream)
    end.synchronize()
    return start.elapsed_time(end)


def autotune(workloads: Sequence, dtype: str = "f32", cache: Optional[str] = None,
             device=None, steps: int = 100, warmup: int = 20,
             tiles: Sequence[Tuple[int, int]] = TILES,
             graph_steps: Sequence[int] = GRAPH_STEPS,
             step_modes: Sequence[int] = STEP_MODES,
             cache_hints: Sequence[int] = CACHE_HINTS,
             lattice_launches: Sequence[int] = LATTICE_LAUNCHES,
             streamings: Sequence[int] = STREAMINGS,
             measure: Optional[Callable] = None) -> dict:
    """Pick the tile shape, step form, cache hints and graph chunk for a batch
    of `workloads`, then the lattice kernel's launch form for that pick.

    Returns {"tile": [tx, ty], "graph_steps": g, "step_mode": m, "cache_hints": c,
    "lattice_launch": w, "streaming": s, "ms_per_step": t, "mlups": ...,
    "candidates": [...], "launch_candidates": [...], "streaming_candidates":
    [...], "device": name, "cached": bool}.  The first stages run with two
    population buffers; the last times in-place streaming at their pick.
    `steps` is rounded up to a multiple of every graph chunk.
    `measure(tile, g, mode, hints, launch=0, streaming=0)` replaces the GPU
    timing (returns ms per step); it exists for tests of the selection and
    caching logic.
    """
    nodes = sum(int(w.nx) * int(w.ny) for w in workloads)
    dev_name = _device_name(device) if measure is None else "measure-callback"
    key = f"{signature(workloads, dtype)}@{dev_name}"
    cached = load_cache(cache).get(key)
    if cached is not None:
        out = dict(cached)
        out["cached"] = True
        return out
    lcm = 1
    for g in graph_steps:
        lcm = lcm * g // _gcd(lcm, g)
    steps = max(lcm, ((int(steps) + lcm - 1) // lcm) * lcm)
    results = []
    for tile in tiles:
        if measure is not None:
            for mode in step_modes:
                for hints in cache_hints:
                    for g in graph_steps:
                        ms = float(measure(tuple(tile), int(g), int(mode), int(hints)))
                        results.append(_record(tile, g, mode, hints, ms, nodes))
            continue
        from . import Batch
        b = Batch(workloads, dtype=dtype, tile=tuple(tile), device=device, graph_steps=0,
                  streaming=0)
        try:
            for mode in step_modes:
                b.set_step_mode(int(mode))
                for hints in cache_hints:
                    b.set_cache_hints(int(hints))
                    for g in graph_steps:
                        b.set_graph_steps(int(g))
                        b.step(max(int(warmup), int(g)))
                        ms = _time_steps(b, steps) / steps
                        results.append(_record(tile, g, b.step_mode, b.cache_hints, ms, nodes))
        finally:
            b.close()
    best = choose(results)
    # second stage: the lattice kernel's launch form at the chosen settings
    launches = []
    for w in lattice_launches:
        if int(w) == 0:
            r = dict(best)
        elif measure is not None:
            ms = float(measure(tuple(best["tile"]), best["graph_steps"], best["step_mode"],
                               best["cache_hints"], launch=int(w)))
            r = _record(best["tile"], best["graph_steps"], best["step_mode"], best["cache_hints"],
                        ms, nodes)
        else:
            from . import Batch
            b = Batch(workloads, dtype=dtype, tile=tuple(best["tile"]), device=device,
                      graph_steps=int(best["graph_steps"]), streaming=0)
            try:
                b.set_step_mode(int(best["step_mode"]))
                b.set_cache_hints(int(best["cache_hints"]))
                b.set_lattice_launch(int(w))
                b.step(max(int(warmup), int(best["graph_steps"])))
                ms = _time_steps(b, steps) / steps
            finally:
                b.close()
            r = _record(best["tile"], best["graph_steps"], best["step_mode"], best["cache_hints"],
                        ms, nodes)
        r["lattice_launch"] = int(w)
        launches.append(r)
    best_launch = choose(launches) if launches else dict(best, lattice_launch=0)
    # last stage: the population streaming (two buffers is the first stages' form)
    streams = []
    for sm in streamings:
        if int(sm) == 0:
            r = dict(best_launch)
        elif measure is not None:
            ms = float(measure(tuple(best["tile"]), best["graph_steps"], best["step_mode"],
                               best["cache_hints"], launch=0, streaming=int(sm)))
            r = _record(best["tile"], best["graph_steps"], best["step_mode"], best["cache_hints"],
                        ms, nodes)
            r["lattice_launch"] = 0
        else:
            from . import Batch
            b = Batch(workloads, dtype=dtype, tile=tuple(best["tile"]), device=device,
                      graph_steps=int(best["graph_steps"]), streaming=int(sm))
            try:
                b.set_step_mode(int(best["step_mode"]))
                b.step(max(int(warmup), int(best["graph_steps"])))
                ms = _time_steps(b, steps) / steps
            finally:
                b.close()
            r = _record(best["tile"], best["graph_steps"], best["step_mode"], best["cache_hints"],
                        ms, nodes)
            r["lattice_launch"] = 0
        r["streaming"] = int(sm)
        streams.append(r)
    pick = choose(streams) if streams else dict(best_launch, streaming=0)
    rec = {"tile": list(best["tile"]), "graph_steps": best["graph_steps"],
           "step_mode": best["step_mode"], "cache_hints": best["cache_hints"],
           "lattice_launch": int(pick["lattice_launch"]), "streaming": int(pick["streaming"]),
           "ms_per_step": pick["ms_per_step"], "mlups": pick["mlups"],
           "candidates": results, "launch_candidates": launches,
           "streaming_candidates": streams, "device": dev_name,
           "nodes": nodes, "instances": len(workloads), "dtype": str(dtype)}
    if cache:
        store_cache(cache, key, rec)
    rec = dict(rec)
    rec["cached"] = False
    return rec


def _record(tile, g, mode, hints, ms, nodes) -> dict:
    return {"tile": [int(tile[0]), int(tile[1])], "graph_steps": int(g), "step_mode": int(mode),
            "cache_hints": int(hints), "ms_per_step": ms,
            "mlups": nodes / (ms * 1e-3) / 1e6 if ms > 0 else float("inf")}


def _gcd(a: int, b: int) -> int:
    while b:
        a, b = b, a % b
    return a


def _device_name(device) -> str:
    import torch
    dev = torch.device(device if device is not None else "cuda")
    return torch.cuda.get_device_name(dev)
