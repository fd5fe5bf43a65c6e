"""Host logic of bench.py (no GPU): the stored HBM-counter figure is reported
only for the kernel source, tile shape and cache hints it was taken with, and
the multi-GPU request is refused."""
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
    monkeypatch.setattr(b, "kernel_source_hash", lambda: rec["kernel_source_sha256_16"])
    assert b.traffic_from_profile(name, tile, hints) == rec["bytes_per_launch"][name]
    other = (64, 4) if tile != (64, 4) else (256, 1)
    assert b.traffic_from_profile(name, other, hints) is None
    assert b.traffic_from_profile(name, tile, 0 if hints else 3) is None
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "0" * 16)
    assert b.traffic_from_profile(name, tile, hints) is None


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
