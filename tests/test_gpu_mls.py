"""The general moving-least-squares transfer (Sec. 2.2, Immersed Boundary
Treatment; Sec. 2.3, nine nodes in a square of side 2.6 dx) on the GPU
against the FP64 oracle, through the C ABI: every weight, both wall modes,
periodic lattices, all tiles, the full-size capillary in FP32; launch forms
and batches bitwise; with the Roma weight and no walls it equals the
default transfer."""
import numpy as np
import pytest

import oracle
import paper_1907_00080_amd as pkg
from workloads import configs

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-mls] {msg}", flush=True)


def with_mls(wl, weight="cubic", h=1.3):
    wl.transfer = "mls"
    wl.mls_weight = weight
    wl.mls_support = h
    return wl


def _vel_err(sim, ref):
    rho, ux, uy = sim.fields()
    du = np.sqrt(np.sum((ux - ref.ux) ** 2 + (uy - ref.uy) ** 2))
    dn = np.sqrt(np.sum(ref.ux ** 2 + ref.uy ** 2))
    return du, dn


def _fp64_side_by_side(wl, schedule, bonds=True):
    sim = pkg.Sim(wl, dtype="f64")
    ref = oracle.Sim(wl)
    for n in schedule:
        sim.step(n - sim.step_count)
        ref.step(n - ref.n)
        du, dn = _vel_err(sim, ref)
        assert du <= 1e-9 * dn + 1e-13, (n, du, dn)
        assert float(np.max(np.abs(sim.all_markers() - ref.all_markers()))) < 1e-9, n
        if bonds:
            assert np.array_equal(sim.bonds(), ref.l2r), n
    sim.close()
    return ref


def adhesive_case():
    from test_gpu_observables import adhesive
    return adhesive()


@pytest.mark.parametrize("weight,h", [("cubic", 1.3), ("gauss", 1.3), ("roma", 1.5),
                                      ("cubic", 1.5), ("gauss", 1.1)])
def test_adhesive_fp64_matches_oracle(weight, h):
    announce(f"adhesive fp64 weight {weight} h {h}")
    ref = _fp64_side_by_side(with_mls(adhesive_case(), weight, h), (1, 10, 40))
    assert int(np.sum(ref.l2r >= 0)) > 0          # bonds formed: wall-side probes exercised


def test_velocity_walls_fp64_matches_oracle():
    announce("velocity walls fp64")
    from test_gpu_walls import bodies_near_walls
    _fp64_side_by_side(with_mls(bodies_near_walls(), "cubic"), (1, 10, 40))


def test_periodic_lattice_fp64_matches_oracle():
    announce("periodic y fp64")
    wl = configs.small_case(nx=64, ny=32, n_rbc=1, periodic_y=1,
                            particles=(configs.PARTICLE_RIGID, configs.PARTICLE_SOFT), seed_offset=53)
    _fp64_side_by_side(with_mls(wl, "gauss"), (1, 15, 50), bonds=False)


@pytest.mark.parametrize("tile", pkg.TILES)
def test_all_tiles_fp32_within_tolerance(tile):
    announce(f"tile {tile} fp32")
    wl = with_mls(configs.small_case(nx=150, ny=36, n_rbc=2,
                                     particles=(configs.PARTICLE_RIGID, configs.PARTICLE_SOFT),
                                     seed_offset=59, mach=0.1))
    sim = pkg.Sim(wl, dtype="f32", tile=tile, graph_steps=10)
    ref = oracle.Sim(wl)
    sim.step(100)
    ref.step(100)
    du, dn = _vel_err(sim, ref)
    assert du <= 1e-5 * dn
    assert float(np.max(np.abs(sim.all_markers() - ref.all_markers()))) < 1e-4
    sim.close()


def test_roma_weight_without_walls_equals_the_default_transfer():
    announce("mls with the roma weight vs the roma kernel, periodic")
    wl = configs.small_case(nx=64, ny=32, n_rbc=1, periodic_y=1,
                            particles=(configs.PARTICLE_RIGID, configs.PARTICLE_SOFT), seed_offset=61)
    a = pkg.Sim(wl, dtype="f64")
    b = pkg.Sim(with_mls(configs.small_case(nx=64, ny=32, n_rbc=1, periodic_y=1,
                                            particles=(configs.PARTICLE_RIGID, configs.PARTICLE_SOFT),
                                            seed_offset=61), "roma"), dtype="f64")
    a.step(30)
    b.step(30)
    for x, y in zip(a.fields(), b.fields()):
        assert np.max(np.abs(x - y)) < 1e-13
    assert np.max(np.abs(a.all_markers() - b.all_markers())) < 1e-12
    a.close()
    b.close()


def test_mls_changes_the_result_next_to_walls():
    # the fit is renormalised over the fluid rows, the kernel truncated: a
    # body touching a wall must see a different result (the switch is live)
    announce("mls vs roma next to a wall")
    a = pkg.Sim(adhesive_case(), dtype="f64")
    b = pkg.Sim(with_mls(adhesive_case(), "roma"), dtype="f64")
    a.step(10)
    b.step(10)
    assert np.max(np.abs(a.all_markers() - b.all_markers())) > 1e-9
    a.close()
    b.close()


def test_capillary_2000x200_full_size_fp32_matches_oracle():
    announce("capillary 2000x200 full size, mls cubic")
    wl = with_mls(configs.capillary_2000x200())
    sim = pkg.Sim(wl, dtype="f32", graph_steps=2)
    ref = oracle.Sim(wl)
    sim.step(3)
    ref.step(3)
    du, dn = _vel_err(sim, ref)
    dx = float(np.max(np.abs(sim.all_markers() - ref.all_markers())))
    announce(f"capillary 2000x200 mls: rel-L2 {du / dn:.3e} markers {dx:.3e}")
    assert du < 1e-5 * dn
    assert dx < 1e-6
    assert np.array_equal(sim.bonds(), ref.l2r)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0 and d["bin_overflow"] == 0
    sim.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_step_forms_bitwise(mode):
    announce(f"step form {mode}")
    wl = with_mls(adhesive_case(), "gauss")
    ref = pkg.Sim(wl, dtype="f32", graph_steps=0)
    ref.set_step_mode(1)
    ref.step(31)
    sim = pkg.Sim(wl, dtype="f32", graph_steps=10)
    sim.set_step_mode(mode)
    sim.step(31)
    for a, b in zip(sim.fields(), ref.fields()):
        assert np.array_equal(a, b)
    assert np.array_equal(sim.all_markers(), ref.all_markers())
    assert np.array_equal(sim.bonds(), ref.bonds())
    sim.close()
    ref.close()


def test_batch_mixing_transfers_equals_single_runs():
    announce("batch, both transfers")
    from test_gpu_observables import adhesive
    ws = [with_mls(adhesive(instance=0), "cubic"), adhesive(nx=80, ny=30, seed=9, instance=1),
          with_mls(configs.small_case(nx=70, ny=28, n_rbc=1, periodic_y=1,
                                      particles=(configs.PARTICLE_SOFT,), seed_offset=67), "gauss", 1.2)]
    ws[2].instance = 2
    batch = pkg.Batch(ws, dtype="f32", graph_steps=10)
    batch.step(30)
    for i, w in enumerate(ws):
        s = pkg.Sim(w, dtype="f32")
        s.step(30)
        for a, b in zip(batch.fields(i), s.fields()):
            assert np.array_equal(a, b), i
        for k in range(len(w.bodies)):
            assert np.array_equal(batch.markers(i, k), s.markers(k)), (i, k)
        s.close()
    batch.close()


def test_adjoint_refuses_the_mls_transfer():
    from paper_1907_00080_amd.adjoint import AdjointWindow
    wl = with_mls(configs.small_case(nx=48, ny=24, n_rbc=1))
    sim = pkg.Sim(wl, dtype="f32")
    with pytest.raises(pkg.LbibError) as e:
        AdjointWindow(sim, 10, 5)
    assert e.value.status == 1
    sim.close()


@pytest.mark.parametrize("weight", ["cubic", "gauss"])
def test_channel_fp32_1000_steps_meets_tolerance(weight):
    """The FP32 bar of the kernel transfer, with the MLS one: 256x64 channel,
    one RBC and one rigid particle, 1000 steps, velocity rel-L2 <= 1e-5 and
    markers <= 1e-4 dx against the FP64 oracle."""
    announce(f"channel 256x64 fp32 1000 steps, mls {weight}")
    wl = with_mls(configs.channel_256x64(), weight)
    sim = pkg.Sim(wl, dtype="f32", graph_steps=100)
    ref = oracle.Sim(wl)
    sim.step(1000)
    ref.step(1000)
    du, dn = _vel_err(sim, ref)
    dx = float(np.max(np.abs(sim.all_markers() - ref.all_markers())))
    announce(f"channel mls {weight}: rel-L2 {du / dn:.3e} markers {dx:.3e}")
    assert du <= 1e-5 * dn
    assert dx <= 1e-4
    sim.close()
