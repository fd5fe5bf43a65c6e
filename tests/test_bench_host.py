"""Host logic of bench.py (no GPU): the stored HBM-counter figure is reported
only for the kernel source, tile shape, streaming form and (with two buffers)
cache hints it was taken with, and the multi-GPU request is refused."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_figure_follows_source_hash_tile_and_hints(monkeypatch):
    b = _bench()
    with open(b.PROFILE_TRAFFIC) as f:
        rec = json.load(f)
    name = "capillary-6667x667"
    tile = tuple(int(v) for v in rec["tiles"][name].split("x"))
    hints = rec["cache_hints"][name]
    st = rec.get("streaming", {}).get(name, 0)
    monkeypatch.setattr(b, "kernel_source_hash", lambda: rec["kernel_source_sha256_16"])
    assert b.traffic_from_profile(name, tile, hints, 0, st) == rec["bytes_per_launch"][name]
    assert b.traffic_from_profile(name, tile, hints, 0, 1 - st) is None
    assert b.traffic_from_profile(name, tile, hints, 4, st) is None   # persistent launch
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "0" * 16)
    assert b.traffic_from_profile(name, tile, hints, 0, st) is None


def test_traffic_lookup_rules(monkeypatch, tmp_path):
    """Synthetic summary: the primary figure and its variants match on tile
    and streaming form; the cache hints count only with two buffers."""
    b = _bench()
    rec = {"kernel_source_sha256_16": "f" * 16, "tiles": {"w": "64x4"}, "cache_hints": {"w": 3},
           "streaming": {"w": 1}, "bytes_per_launch": {"w": 100},
           "variants": [{"workload": "w", "tile": "32x8", "cache_hints": 3, "streaming": 1,
                         "bytes_per_launch": 101},
                        {"workload": "w", "tile": "64x4", "cache_hints": 0, "streaming": 0,
                         "bytes_per_launch": 102},
                        {"workload": "v", "tile": "64x4", "cache_hints": 0, "streaming": 0,
                         "bytes_per_launch": 103}]}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(b, "PROFILE_TRAFFIC", str(path))
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "f" * 16)
    assert b.traffic_from_profile("w", (64, 4), 3, 0, 1) == 100
    assert b.traffic_from_profile("w", (64, 4), 0, 0, 1) == 100     # hints unused in place
    assert b.traffic_from_profile("w", (32, 8), 0, 0, 1) == 101
    assert b.traffic_from_profile("w", (64, 4), 0, 0, 0) == 102
    assert b.traffic_from_profile("w", (64, 4), 3, 0, 0) is None    # two buffers: hints count
    assert b.traffic_from_profile("w", (256, 1), 3, 0, 1) is None
    assert b.traffic_from_profile("v", (64, 4), 0, 0, 0) == 103
    assert b.traffic_from_profile("u", (64, 4), 0, 0, 0) is None


def test_stored_counters_match_current_kernel():
    """The committed counter figures were taken with the current fused kernel."""
    b = _bench()
    with open(b.PROFILE_TRAFFIC) as f:
        rec = json.load(f)
    assert rec["kernel_source_sha256_16"] == b.kernel_source_hash()


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_graph_chunk_covers_the_timed_region():
    """The timed region is replayed from graphs for any step count: the chunk
    shrinks to the region (even, for the two population buffers)."""
    b = _bench()
    assert b.graph_chunk(100, 2000) == 100
    assert b.graph_chunk(100, 20) == 20
    assert b.graph_chunk(100, 25) == 24
    assert b.graph_chunk(100, 1) == 0
