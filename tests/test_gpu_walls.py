"""Zou-He velocity walls on the node rows (the paper's wall condition, Sec.
2.1) on the GPU against the FP64 oracle, through the C ABI: Couette and
forced Poiseuille flow, bodies and bonds next to the walls, the adhesion box
with a moving top wall; launch forms and batches bitwise."""
import numpy as np
import pytest

import oracle
import paper_1907_00080_amd as pkg
from workloads import configs, geometry

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-walls] {msg}", flush=True)


def _vel_err(sim, ref):
    rho, ux, uy = sim.fields()
    du = np.sqrt(np.sum((ux - ref.ux) ** 2 + (uy - ref.uy) ** 2))
    dn = np.sqrt(np.sum(ref.ux ** 2 + ref.uy ** 2))
    return du, dn, float(np.max(np.abs(rho - ref.rho)))


def lattice_case(kind, nx=70, ny=23, tau=0.8):
    if kind == "couette":
        return configs.Workload("couette", nx, ny, tau, walls="zou-he", u_wall=(0.004, -0.011))
    rng = np.random.default_rng(ny)
    u0 = 0.01 * rng.standard_normal((2, ny, nx))
    return configs.Workload("poiseuille", nx, ny, tau, gx=3e-6, gy=-1e-6, walls="zou-he",
                            u_wall=(0.0, 0.0), u0=u0)


@pytest.mark.parametrize("kind", ["couette", "poiseuille"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_lattice_with_velocity_walls_matches_oracle(kind, dtype, tol):
    announce(f"lattice {kind} {dtype}")
    wl = lattice_case(kind)
    sim = pkg.Sim(wl, dtype=dtype)
    ref = oracle.Sim(wl)
    for n in (1, 9, 120):
        sim.step(n - sim.step_count)
        ref.step(n - ref.n)
        du, dn, drho = _vel_err(sim, ref)
        assert du <= tol * dn + 1e-14, (n, du, dn)
        assert drho < (1e-13 if dtype == "f64" else 1e-6)
    sim.close()


@pytest.mark.parametrize("tile", pkg.TILES)
def test_couette_all_tiles_fp32(tile):
    announce(f"couette tile {tile}")
    wl = lattice_case("couette", nx=300, ny=50, tau=1.0)
    sim = pkg.Sim(wl, dtype="f32", tile=tile)
    ref = oracle.Sim(wl)
    sim.step(200)
    ref.step(200)
    du, dn, _ = _vel_err(sim, ref)
    assert du <= 1e-5 * dn
    sim.close()


def bodies_near_walls():
    """A red cell mid-channel, a soft adhesive particle touching the lower
    wall row and a rigid adhesive one at the moving upper wall."""
    nx, ny = 96, 40
    r = 4.0
    soft = geometry.place(geometry.circle(r, 30), 0.2, [30.0, 0.0])
    soft[:, 1] += 0.25 - soft[:, 1].min()
    rig = geometry.place(geometry.circle(r, 30), 0.1, [70.0, 0.0])
    rig[:, 1] += (ny - 1 - 0.25) - rig[:, 1].max()
    cell = geometry.place(geometry.rbc_contour(8.0, 60), 0.3, [60.0, 20.0])
    ks = 2e-2
    adh = configs.Adhesion(y_cr=1.0, y_eq=0.5, kf0_dt=0.2, kr0_dt=0.01, sigma_ts_frac=0.5,
                           kbt=1e-3)
    u_top = 0.01
    y = np.arange(ny, dtype=np.float64)
    u0 = np.zeros((2, ny, nx))
    u0[0] = (u_top * y / (ny - 1))[:, None]
    return configs.Workload(
        "walls-bodies", nx, ny, 1.0, seed=configs.SEED_BASE + 31,
        bodies=[configs.Body(configs.PARTICLE_SOFT, soft, ks=ks, kb=0.05 * ks * r * r,
                             sigma=5e-3, ligand_stride=2),
                configs.Body(configs.PARTICLE_RIGID, rig, sigma=8e-3, ligand_stride=2),
                configs.Body(configs.RBC_KINEMATIC, cell, ks=ks, kb=0.001)],
        receptors=configs.uniform_receptors(nx), adhesion=adh, u0=u0,
        walls="zou-he", u_wall=(0.0, u_top))


def test_bodies_and_bonds_next_to_velocity_walls_fp64():
    announce("bodies near velocity walls fp64")
    wl = bodies_near_walls()
    sim = pkg.Sim(wl, dtype="f64")
    ref = oracle.Sim(wl)
    for n in (1, 10, 40):
        sim.step(n - sim.step_count)
        ref.step(n - ref.n)
        du, dn, _ = _vel_err(sim, ref)
        assert du <= 1e-9 * dn + 1e-13, (n, du, dn)
        assert float(np.max(np.abs(sim.all_markers() - ref.all_markers()))) < 1e-9
        assert np.array_equal(sim.bonds(), ref.l2r)
    assert int(np.sum(ref.l2r >= 0)) > 0          # bonds formed against both walls' geometry
    sim.close()


@pytest.mark.parametrize("kind", [configs.PARTICLE_RIGID, configs.PARTICLE_SOFT])
def test_couette_box_small_fp64_matches_oracle(kind):
    announce(f"couette box kind {kind}")
    wl = configs.couette_box(kind=kind, nx=120, ny=40, dx_um=0.075)
    wl.adhesion.kf0_dt = 0.2
    sim = pkg.Sim(wl, dtype="f64")
    ref = oracle.Sim(wl)
    for n in (1, 30, 100):
        sim.step(n - sim.step_count)
        ref.step(n - ref.n)
        du, dn, _ = _vel_err(sim, ref)
        assert du <= 1e-9 * dn + 1e-13, (n, du, dn)
        assert float(np.max(np.abs(sim.all_markers() - ref.all_markers()))) < 1e-9
        assert np.array_equal(sim.bonds(), ref.l2r)
    sim.close()


def test_couette_box_full_size_fp32_runs_clean():
    announce("couette box 600x200 fp32")
    wl = configs.couette_box()
    sim = pkg.Sim(wl, dtype="f32", graph_steps=100)
    sim.step(2000)
    d = sim.diagnostics()
    assert d["nonfinite"] == 0 and d["bin_overflow"] == 0 and d["sync_timeouts"] == 0
    rho, ux, uy = sim.fields()
    # away from the particle the flow stays the Couette line of the moving wall
    far = ux[:, int(0.75 * wl.nx)]
    y = np.arange(wl.ny)
    assert np.max(np.abs(far - wl.u_wall[1] * y / (wl.ny - 1))) < 0.05 * wl.u_wall[1]
    sim.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_step_forms_bitwise_with_velocity_walls(mode):
    announce(f"step form {mode}")
    wl = bodies_near_walls()
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


def test_batch_mixing_wall_modes_equals_single_runs():
    announce("batch, both wall modes")
    ws = [bodies_near_walls(), configs.small_case(nx=80, ny=30, n_rbc=1,
                                                  particles=(configs.PARTICLE_SOFT,), seed_offset=41),
          lattice_case("couette", nx=64, ny=20)]
    for i, w in enumerate(ws):
        w.instance = i
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


def test_adjoint_refuses_velocity_walls():
    from paper_1907_00080_amd.adjoint import AdjointWindow
    sim = pkg.Sim(lattice_case("couette"), dtype="f32")
    with pytest.raises(pkg.LbibError) as e:
        AdjointWindow(sim, 10, 5)
    assert e.value.status == 1
    sim.close()
