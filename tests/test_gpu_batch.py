"""Batched sweeps on the GPU (many uneven instances advanced together).

A batch must give every instance exactly the result it gets when run on its
own (bitwise: the instances share launches, never arithmetic), for every tile
shape and with graph-captured chunks; and each instance must match the FP64
oracle to the same bar as a single run.
"""
import numpy as np
import pytest

import oracle
import paper_1907_00080_amd as pkg
from paper_1907_00080_amd.tune import autotune
from workloads import configs, geometry

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-batch] {msg}", flush=True)


def _adhesive(nx, ny, seed, instance):
    r = 3.0
    xy = geometry.place(geometry.circle(r, 24), 0.1, [20.0, r - 0.2])
    xy2 = geometry.place(geometry.circle(r, 24), 0.3, [44.0, ny - 1 - r + 0.25])
    ks = 2e-2
    bodies = [configs.Body(configs.PARTICLE_SOFT, xy, ks=ks, kb=0.05 * ks * r * r, sigma=5e-3,
                           ligand_stride=2),
              configs.Body(configs.PARTICLE_RIGID, xy2, sigma=8e-3, ligand_stride=2)]
    g = configs.poiseuille_force(0.01, ny, 1.0)
    rho0, u0 = configs.poiseuille_init(nx, ny, g, 1.0)
    adh = configs.Adhesion(y_cr=1.0, y_eq=0.5, kf0_dt=0.2, kr0_dt=0.01, sigma_ts_frac=0.5,
                           kbt=1e-3)
    w = configs.Workload(f"adh{instance}", nx, ny, 1.0, gx=g, seed=configs.SEED_BASE + seed,
                         bodies=bodies, receptors=configs.uniform_receptors(nx), adhesion=adh,
                         rho0=rho0, u0=u0)
    w.instance = instance
    return w


def uneven_instances():
    """Five instances of different sizes and contents: red cells, rigid and
    soft particles, adhesion with bonds, a periodic box, a ragged last tile."""
    ws = [configs.small_case(nx=96, ny=24, n_rbc=1, seed_offset=21),
          configs.small_case(nx=80, ny=30, n_rbc=0,
                             particles=(configs.PARTICLE_RIGID, configs.PARTICLE_SOFT),
                             seed_offset=22),
          _adhesive(64, 24, 7, 2),
          configs.small_case(nx=72, ny=40, n_rbc=1, particles=(configs.PARTICLE_SOFT,),
                             periodic_y=1, seed_offset=23),
          configs.small_case(nx=129, ny=33, n_rbc=2, particles=(configs.PARTICLE_RIGID,),
                             seed_offset=24)]
    for i, w in enumerate(ws):
        if i != 2:
            w.instance = i
    return ws


def _same_as_single(batch, i, w, single):
    for a, b in zip(batch.fields(i), single.fields()):
        assert np.array_equal(a, b), (i, "fields")
    for k in range(len(w.bodies)):
        assert np.array_equal(batch.markers(i, k), single.markers(k)), (i, k)
    assert np.array_equal(batch.bonds(i), single.bonds()), (i, "bonds")


@pytest.mark.parametrize("tile", pkg.TILES)
def test_batch_bitwise_equals_individual_runs(tile):
    announce(f"batch vs single runs, tile {tile}")
    ws = uneven_instances()
    batch = pkg.Batch(ws, dtype="f32", tile=tile, graph_steps=10)
    batch.step(60)
    d = batch.diagnostics()
    assert d["nonfinite"] == 0 and d["bin_overflow"] == 0 and d["sync_timeouts"] == 0
    bonded = 0
    for i, w in enumerate(ws):
        s = pkg.Sim(w, dtype="f32", tile=tile)
        s.step(60)
        _same_as_single(batch, i, w, s)
        bonded += int(np.sum(s.bonds() >= 0))
        s.close()
    batch.close()
    assert bonded > 0       # the adhesive instance formed bonds


@pytest.mark.parametrize("tile", [(64, 4), (256, 1)])
def test_persistent_lattice_launch_is_bitwise_the_default(tile):
    """The lattice kernel's persistent launch (a fixed grid of 1, 2 or 8
    workgroups per CU walking the tiles) gives the one-workgroup-per-tile
    launch's bits: on the uneven batch and on the 2000 x 200 capillary."""
    announce(f"persistent lattice launch, tile {tile}")
    ws = uneven_instances()
    ref = pkg.Batch(ws, dtype="f32", tile=tile, graph_steps=10)
    ref.step(40)
    for wpc in (1, 2, 8):
        b = pkg.Batch(ws, dtype="f32", tile=tile, graph_steps=10)
        b.set_lattice_launch(wpc)
        assert b.lattice_launch == wpc
        b.step(40)
        d = b.diagnostics()
        assert d["nonfinite"] == 0 and d["bin_overflow"] == 0
        for i, w in enumerate(ws):
            for x, y in zip(b.fields(i), ref.fields(i)):
                assert np.array_equal(x, y), (wpc, i)
            for k in range(len(w.bodies)):
                assert np.array_equal(b.markers(i, k), ref.markers(i, k)), (wpc, i, k)
        b.close()
    ref.close()
    wl = configs.capillary_2000x200()
    runs = []
    for wpc in (0, 4):
        s = pkg.Sim(wl, dtype="f32", tile=tile, graph_steps=10)
        s.set_lattice_launch(wpc)
        s.step(20)
        runs.append((s.fields(), s.all_markers()))
        s.close()
    for x, y in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(x, y)
    assert np.array_equal(runs[0][1], runs[1][1])


def test_batch_fp64_matches_oracle_per_instance():
    announce("batch fp64 vs oracle")
    ws = uneven_instances()
    batch = pkg.Batch(ws, dtype="f64", graph_steps=0)
    refs = [oracle.Sim(w) for w in ws]
    for n in (1, 25):
        batch.step(n - batch.step_count)
        for i, (w, r) in enumerate(zip(ws, refs)):
            r.step(n - r.n)
            rho, ux, uy = batch.fields(i)
            du = np.sqrt(np.sum((ux - r.ux) ** 2 + (uy - r.uy) ** 2))
            dn = np.sqrt(np.sum(r.ux ** 2 + r.uy ** 2))
            # (an instance at rest has dn = 0: round-off of the rest state then bounds du)
            assert du <= 1e-9 * dn + 1e-13, (i, n, du, dn)
            for k in range(len(w.bodies)):
                assert np.max(np.abs(batch.markers(i, k) - r.bodies[k].X)) < 1e-9, (i, k, n)
            assert np.array_equal(batch.bonds(i), r.l2r), (i, n)
    batch.close()


def test_sweep_full_size_sampled():
    """The 64-instance sweep (20-100 um long capillaries, 15.6 M nodes) as
    one batch: sampled instances equal their single runs bitwise, and one
    matches the oracle."""
    ws = configs.sweep_instances(64)
    announce(f"sweep of {len(ws)} instances, {sum(w.nodes for w in ws)} nodes")
    for tile, g in (((64, 4), 10), ((256, 1), 2)):
        announce(f"sweep tile {tile} graphs of {g}")
        batch = pkg.Batch(ws, dtype="f32", tile=tile, graph_steps=g)
        batch.step(4)
        d = batch.diagnostics()
        assert d["nonfinite"] == 0 and d["bin_overflow"] == 0 and d["sync_timeouts"] == 0
        for i in (0, 17, 63):
            s = pkg.Sim(ws[i], dtype="f32", tile=tile)
            s.step(4)
            _same_as_single(batch, i, ws[i], s)
            s.close()
        if tile == (64, 4):
            i = 5
            r = oracle.Sim(ws[i])
            r.step(4)
            rho, ux, uy = batch.fields(i)
            du = np.sqrt(np.sum((ux - r.ux) ** 2 + (uy - r.uy) ** 2))
            dn = np.sqrt(np.sum(r.ux ** 2 + r.uy ** 2))
            announce(f"sweep instance {i} vs oracle: rel-L2 {du / dn:.3e}")
            assert du / dn < 1e-5
            for k in range(len(ws[i].bodies)):
                assert np.max(np.abs(batch.markers(i, k) - r.bodies[k].X)) < 1e-6
            assert np.array_equal(batch.bonds(i), r.l2r)
        batch.close()


def test_autotune_picks_a_candidate_and_caches(tmp_path):
    announce("autotune")
    ws = uneven_instances()[:3]
    path = str(tmp_path / "tune.json")
    rec = autotune(ws, "f32", cache=path, steps=20, warmup=10)
    assert rec["cached"] is False
    assert tuple(rec["tile"]) in pkg.TILES and rec["graph_steps"] in (10, 100)
    assert len(rec["candidates"]) == len(pkg.TILES) * 2 * 3 * 3   # tiles x graph chunks x forms x hints
    assert rec["step_mode"] in (1, 2, 3)
    # the launch stage starts from the first stage's best and keeps the fastest form
    launches = rec["launch_candidates"]
    assert [c["lattice_launch"] for c in launches] == [0, 1, 2, 4, 8]
    assert launches[0]["ms_per_step"] == min(c["ms_per_step"] for c in rec["candidates"])
    assert rec["lattice_launch"] in (0, 1, 2, 4, 8)
    # then the streaming form: two buffers (the launch stage's best) or in place
    streams = rec["streaming_candidates"]
    assert [c["streaming"] for c in streams] == [0, 1]
    assert streams[0]["ms_per_step"] == min(c["ms_per_step"] for c in launches)
    assert rec["ms_per_step"] == min(c["ms_per_step"] for c in streams)
    again = autotune(ws, "f32", cache=path, steps=20, warmup=10)
    assert again["cached"] is True
    assert again["tile"] == rec["tile"] and again["graph_steps"] == rec["graph_steps"]
