"""Selection and caching logic of the batch autotuner (host only, no GPU)."""
import json

from paper_1907_00080_amd import tune
from workloads import configs


def _ws():
    return [configs.small_case(nx=48, ny=24, n_rbc=1, seed_offset=31),
            configs.small_case(nx=64, ny=20, n_rbc=0, seed_offset=32)]


def test_signature_is_stable_and_sensitive():
    a, b = _ws(), _ws()
    assert tune.signature(a, "f32") == tune.signature(b, "f32")
    assert tune.signature(a, "f32") != tune.signature(a, "f64")
    assert tune.signature(a, "f32") != tune.signature(a[:1], "f32")
    c = _ws()
    c[1] = configs.small_case(nx=65, ny=20, n_rbc=0, seed_offset=32)
    assert tune.signature(a, "f32") != tune.signature(c, "f32")
    # everything that changes which kernel variants and step forms run
    for attr, val in (("walls", "zou-he"), ("transfer", "mls"), ("repulsion", 1e-5)):
        d = _ws()
        setattr(d[0], attr, val)
        assert tune.signature(d, "f32") != tune.signature(a, "f32"), attr
    e, f = _ws(), _ws()
    for w, weight in ((e[0], "cubic"), (f[0], "gauss")):
        w.transfer, w.mls_weight = "mls", weight
    assert tune.signature(e, "f32") != tune.signature(f, "f32")


def test_choose_fastest_and_first_on_ties():
    rs = [{"tile": [64, 4], "graph_steps": 10, "ms_per_step": 2.0},
          {"tile": [32, 8], "graph_steps": 10, "ms_per_step": 1.0},
          {"tile": [256, 1], "graph_steps": 100, "ms_per_step": 1.0}]
    assert tune.choose(rs)["tile"] == [32, 8]


def test_autotune_selects_minimum_and_caches(tmp_path):
    calls = []
    cost = {((64, 4), 10): 3.0, ((64, 4), 100): 2.5, ((128, 2), 10): 2.9,
            ((128, 2), 100): 1.5, ((32, 8), 10): 4.0, ((32, 8), 100): 1.7,
            ((256, 1), 10): 2.2, ((256, 1), 100): 2.0}

    def measure(tile, g, mode, hints, launch=0, streaming=0):
        calls.append((tile, g, mode, hints, launch, streaming))
        return (cost[(tile, g)] + (0.0 if mode == 2 else 0.25 * mode) + (0.0 if hints == 1 else 0.1)
                - (0.1 if launch == 4 else 0.0) - (0.2 if streaming else 0.0))

    path = str(tmp_path / "sub" / "tune.json")
    ws = _ws()
    rec = tune.autotune(ws, "f32", cache=path, measure=measure)
    assert rec["tile"] == [128, 2] and rec["graph_steps"] == 100 and not rec["cached"]
    assert rec["step_mode"] == 2 and rec["cache_hints"] == 1
    # second stage: the launch forms at that pick (0 is the first stage's own time)
    assert len(calls) == 72 + 4 + 1 and all(c[4] == 0 and c[5] == 0 for c in calls[:72])
    assert [c[4] for c in calls[72:76]] == [1, 2, 4, 8]
    assert all(c[:4] == ((128, 2), 100, 2, 1) for c in calls[72:])
    assert calls[76][4:] == (0, 1)   # in place, at the pick, with the per-tile launch
    assert len(rec["launch_candidates"]) == 5 and len(rec["streaming_candidates"]) == 2
    # in place (1.5 - 0.2) beats the best two-buffer launch form (1.5 - 0.1)
    assert rec["streaming"] == 1 and rec["lattice_launch"] == 0
    nodes = sum(w.nodes for w in ws)
    assert abs(rec["ms_per_step"] - 1.3) < 1e-12
    assert abs(rec["mlups"] - nodes / 1.3e-3 / 1e6) < 1e-9
    with open(path) as f:
        data = json.load(f)
    assert len(data) == 1
    again = tune.autotune(ws, "f32", cache=path, measure=measure)
    assert again["cached"] and again["tile"] == [128, 2] and again["streaming"] == 1
    assert len(calls) == 77
    # another batch adds a second record and keeps the first
    tune.autotune(ws[:1], "f32", cache=path, measure=measure)
    with open(path) as f:
        assert len(json.load(f)) == 2


def test_autotune_without_cache_measures_every_time():
    n = []
    tune.autotune(_ws(), "f32", cache=None,
                  measure=lambda t, g, m, c, launch=0, streaming=0: n.append(1) or 1.0)
    rec = tune.autotune(_ws(), "f32", cache=None,
                        measure=lambda t, g, m, c, launch=0, streaming=0: n.append(1) or 1.0)
    assert len(n) == 2 * (72 + 4 + 1)
    # ties go to the earlier candidate: one workgroup per tile, two buffers
    assert rec["lattice_launch"] == 0 and rec["streaming"] == 0
