"""Vertex repulsion between bodies (Sec. 2.2, Eq. repFor) on the GPU, against
the FP64 oracle, called through the C ABI.

Fixtures crowd red cells, rigid and soft particles to about one lattice unit
apart, with bodies across the periodic x seam (a 129-wide lattice whose last
64-wide tile is one column wide) and, in a periodic box, across the y seam.
The bar is the one of the other body tests: FP64 to round-off (1e-9), FP32
within the channel tolerances, bitwise agreement between launch forms.
"""
import numpy as np
import pytest

import oracle
import paper_1907_00080_amd as pkg
from oracle import repulsion as orep
from workloads import configs, geometry

pytestmark = pytest.mark.gpu

C = configs.REPULSION_COEFF


def announce(msg):
    print(f"[gpu-repulsion] {msg}", flush=True)


def crowd(coeff=C, nx=129, ny=40):
    """Red cells and particles with gaps of about one lattice unit; one red
    cell and a rigid particle face each other across the x seam."""
    ks = 0.02
    cell_a = geometry.place(geometry.rbc_contour(8.0, 60), 0.0, [30.0, 20.0])
    right = float(np.max(cell_a[:, 0]))
    rig = geometry.place(geometry.circle(3.0, 24), 0.0, [right + 3.0 + 1.1, 20.0])
    soft = geometry.place(geometry.circle(4.0, 30), 0.2, [right + 3.0 + 1.1, 20.0 + 3.0 + 4.0 + 1.0])
    cell_b = geometry.place(geometry.rbc_contour(8.0, 60), 0.3, [3.0, 15.0])
    left = float(np.min(cell_b[:, 0]))
    rig2 = geometry.place(geometry.circle(3.0, 24), 0.4, [left - 3.0 - 1.2 + nx, 15.0])
    g = configs.poiseuille_force(0.02, ny, 1.0)
    rho0, u0 = configs.poiseuille_init(nx, ny, g, 1.0)
    bodies = [configs.Body(configs.RBC_KINEMATIC, cell_a, ks=ks, kb=0.001),
              configs.Body(configs.PARTICLE_RIGID, rig),
              configs.Body(configs.PARTICLE_SOFT, soft, ks=ks, kb=0.05 * ks * 16),
              configs.Body(configs.RBC_KINEMATIC, cell_b, ks=ks, kb=0.001),
              configs.Body(configs.PARTICLE_RIGID, rig2)]
    return configs.Workload("crowd", nx, ny, 1.0, gx=g, bodies=bodies, rho0=rho0, u0=u0,
                            repulsion=coeff, repulsion_cutoff=2.0)


def periodic_pair(coeff=C):
    """Two particles facing each other across the y seam of a periodic box."""
    nx, ny = 80, 30
    a = geometry.place(geometry.circle(3.0, 24), 0.0, [40.0, 3.5])
    b = geometry.place(geometry.circle(3.0, 24), 0.1, [40.3, 26.5 - 0.1])
    ks = 0.02
    return configs.Workload("ypair", nx, ny, 1.0, gx=1e-6, gy=-2e-6, periodic_y=1,
                            bodies=[configs.Body(configs.PARTICLE_RIGID, a),
                                    configs.Body(configs.PARTICLE_SOFT, b, ks=ks, kb=0.05 * ks * 9)],
                            repulsion=coeff, repulsion_cutoff=2.0)


def _close_pairs(wl):
    mags = orep.magnitudes([b.xy for b in wl.bodies], 1.0, wl.repulsion_cutoff, wl.nx, wl.ny,
                           bool(wl.periodic_y))
    return [int(np.count_nonzero(m)) for m in mags]


def _compare(sim, ref, n_list, tol=1e-9):
    for n in n_list:
        sim.step(n - sim.step_count)
        ref.step(n - ref.n)
        rho, ux, uy = sim.fields()
        du = np.sqrt(np.sum((ux - ref.ux) ** 2 + (uy - ref.uy) ** 2))
        dn = np.sqrt(np.sum(ref.ux ** 2 + ref.uy ** 2))
        assert du <= tol * dn + 1e-13, (n, du, dn)
        dx = float(np.max(np.abs(sim.all_markers() - ref.all_markers())))
        assert dx < tol, (n, dx)
        scale = max(np.max(np.abs(f)) for f in ref.marker_force)
        for b in range(len(ref.bodies)):
            assert np.max(np.abs(sim.marker_forces(b) - ref.marker_force[b])) <= tol * scale + 1e-13


def test_fixtures_have_close_pairs():
    # every body of the crowd except the far soft particle has vertices within
    # the cutoff of another body; both bodies of the periodic pair do
    c = _close_pairs(crowd())
    assert c[0] > 0 and c[1] > 0 and c[3] > 0 and c[4] > 0
    assert all(k > 0 for k in _close_pairs(periodic_pair()))


@pytest.mark.parametrize("tile", pkg.TILES)
def test_crowd_fp64_matches_oracle(tile):
    announce(f"crowd fp64 tile {tile}")
    wl = crowd()
    sim = pkg.Sim(wl, dtype="f64", tile=tile)
    assert sim.step_mode != 2          # the merged form is off with the repulsion
    _compare(sim, oracle.Sim(wl), (1, 10, 40))
    assert sim.diagnostics()["bin_overflow"] == 0
    sim.close()


def test_strong_repulsion_fp64_matches_oracle():
    # a hundred times the paper's coefficient: the repulsion dominates the motion
    announce("crowd fp64, 100x coefficient")
    wl = crowd(coeff=100.0 * C)
    sim = pkg.Sim(wl, dtype="f64")
    _compare(sim, oracle.Sim(wl), (1, 20, 60))
    sim.close()


def test_periodic_y_pair_fp64_matches_oracle():
    announce("periodic-y pair fp64")
    wl = periodic_pair(coeff=100.0 * C)
    sim = pkg.Sim(wl, dtype="f64", tile=(128, 2))
    _compare(sim, oracle.Sim(wl), (1, 15, 50))
    sim.close()


def test_repulsion_is_applied_on_the_gpu():
    announce("repulsion changes the trajectory")
    on = pkg.Sim(crowd(), dtype="f64")
    off = pkg.Sim(crowd(coeff=0.0), dtype="f64")
    on.step(10)
    off.step(10)
    d = float(np.max(np.abs(on.all_markers() - off.all_markers())))
    assert d > 1e-6, d
    # the red cell next to the rigid particle spreads a different force
    assert np.max(np.abs(on.marker_forces(0) - off.marker_forces(0))) > 1e-6
    on.close()
    off.close()


def test_crowd_fp32_meets_tolerance():
    announce("crowd fp32 200 steps")
    wl = crowd()
    sim = pkg.Sim(wl, dtype="f32", graph_steps=10)
    ref = oracle.Sim(wl)
    sim.step(200)
    ref.step(200)
    rho, ux, uy = sim.fields()
    du = np.sqrt(np.sum((ux - ref.ux) ** 2 + (uy - ref.uy) ** 2))
    dn = np.sqrt(np.sum(ref.ux ** 2 + ref.uy ** 2))
    assert du / dn < 1e-5
    assert float(np.max(np.abs(sim.all_markers() - ref.all_markers()))) < 1e-4
    sim.close()


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_launch_forms_bitwise_identical(mode):
    announce(f"bitwise eager/graph, step mode {mode}")
    wl = crowd(coeff=100.0 * C)
    ref = pkg.Sim(wl, dtype="f32", graph_steps=0)
    ref.step(33)
    sim = pkg.Sim(wl, dtype="f32", graph_steps=10)
    sim.set_step_mode(mode)
    assert sim.step_mode in (1, 3)
    sim.step(33)
    for a, b in zip(sim.fields(), ref.fields()):
        assert np.array_equal(a, b)
    assert np.array_equal(sim.all_markers(), ref.all_markers())
    d = sim.diagnostics()
    assert d["bin_overflow"] == 0 and d["sync_timeouts"] == 0
    sim.close()
    ref.close()


@pytest.mark.parametrize("tile", [(64, 4), (256, 1)])
def test_batch_bitwise_equals_single_runs(tile):
    announce(f"batch with repulsion, tile {tile}")
    ws = [crowd(coeff=100.0 * C), periodic_pair(coeff=100.0 * C), crowd(coeff=0.0, nx=96)]
    for i, w in enumerate(ws):
        w.instance = i
    batch = pkg.Batch(ws, dtype="f32", tile=tile, graph_steps=10)
    batch.step(40)
    for i, w in enumerate(ws):
        s = pkg.Sim(w, dtype="f32", tile=tile)
        s.step(40)
        for a, b in zip(batch.fields(i), s.fields()):
            assert np.array_equal(a, b), i
        for k in range(len(w.bodies)):
            assert np.array_equal(batch.markers(i, k), s.markers(k)), (i, k)
        s.close()
    batch.close()


def test_adjoint_refuses_repulsion():
    from paper_1907_00080_amd.adjoint import AdjointWindow
    sim = pkg.Sim(periodic_pair(), dtype="f32")
    with pytest.raises(pkg.LbibError) as e:
        AdjointWindow(sim, 10, 5)
    assert e.value.status == 1
    sim.close()
