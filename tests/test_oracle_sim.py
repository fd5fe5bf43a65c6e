"""Whole-step pins of the oracle (Sec. 2.3 order of operations, Sec. 3 set-up).

Special cases whose outcome is fixed without running the method: a
stress-free cell in fluid at rest stays put; a stressed cell in a periodic
box cannot create momentum; force-free markers in the steady channel flow
move by the interpolated closed-form velocity every step; a rigid particle
in fluid at rest stays at rest and in uniform flow is carried along.
"""
import numpy as np
import pytest

import oracle
from oracle import ib, lattice
from workloads import configs, geometry


def _wl(nx, ny, bodies, g=0.0, periodic_y=0, u0=None, rho0=None):
    return configs.Workload("t", nx, ny, 1.0, gx=g, periodic_y=periodic_y, bodies=bodies,
                            u0=u0, rho0=rho0)


def test_unstressed_cell_in_rest_fluid_is_fixed():
    xy = geometry.place(geometry.rbc_contour(6.0, 40), 0.3, [12.0, 9.5])
    wl = _wl(24, 20, [configs.Body(configs.RBC_KINEMATIC, xy, ks=0.03, kb=0.002)])
    s = oracle.Sim(wl)
    s.step(20)
    # only the rounding of the BDF2 update itself remains
    assert np.max(np.abs(s.bodies[0].X - xy)) < 1e-12
    assert np.max(np.abs(s.ux)) < 1e-15 and np.max(np.abs(s.uy)) < 1e-15


def test_stressed_cell_periodic_box_conserves_mass_and_momentum():
    rng = np.random.default_rng(0)
    xy = geometry.place(geometry.rbc_contour(6.0, 40), 0.3, [12.0, 9.5])
    pert = xy + 0.3 * rng.standard_normal(xy.shape)
    wl = _wl(24, 20, [configs.Body(configs.RBC_KINEMATIC, xy, ks=0.03, kb=0.002)], periodic_y=1)
    s = oracle.Sim(wl)
    s.bodies[0].X = pert.copy()
    s.bodies[0].Xm = pert.copy()
    m0 = s.f.sum()
    moved = 0.0
    for _ in range(30):
        s.step(1)
        assert abs(s.f.sum() - m0) < 1e-11
        assert abs((s.rho * s.ux).sum()) < 1e-13 and abs((s.rho * s.uy).sum()) < 1e-13
        moved = max(moved, np.max(np.abs(s.bodies[0].X - pert)))
    assert moved > 1e-3   # the stressed cell does relax


def test_passive_markers_follow_steady_channel_flow():
    nx, ny, tau = 8, 12, 1.0
    g = 1e-5
    prof = configs.poiseuille_profile(g, ny, tau)
    rho0, u0 = configs.poiseuille_init(nx, ny, g, tau)
    # bring the fluid to its exact discrete steady state first
    f = lattice.equilibrium(rho0, u0[0], u0[1])
    F = np.zeros((2, ny, nx))
    F[0] = g
    for _ in range(4000):
        f, *_ = lattice.lb_step(f, F[0], F[1], tau)
    xy = np.array([[1.3, 3.37], [4.0, 5.5], [6.6, 8.0], [2.2, 2.81]])
    wl = _wl(nx, ny, [configs.Body(configs.RBC_KINEMATIC, xy[[0, 1, 2, 3]], ks=0.0, kb=0.0, ka=0.0)], g=g)
    s = oracle.Sim(wl)
    s.f = f
    X0 = s.bodies[0].X.copy()
    # interpolated closed form: u(Y) + u''/2 m2(Y), u'' = -g/nu
    Y = X0[:, 1]
    jj = np.floor(Y + 0.5)[:, None] + np.arange(-1, 2)[None, :]
    m2 = (ib.phi(jj - Y[:, None]) * (jj - Y[:, None]) ** 2).sum(1)
    nu = (tau - 0.5) / 3
    yy = Y
    U = g / (2 * nu) * ((yy + 0.5) * (ny - 0.5 - yy) + (16 * 0.25 - 3) / 12) - 0.5 * g / nu * m2
    for n in range(1, 11):
        s.step(1)
        assert np.allclose(s.bodies[0].X[:, 0], X0[:, 0] + n * U, atol=1e-12)
        assert np.allclose(s.bodies[0].X[:, 1], Y, atol=1e-13)
    assert prof.max() > 0


def _rigid_particle(center, r=3.0, n=24):
    return configs.Body(configs.PARTICLE_RIGID, geometry.place(geometry.circle(r, n), 0.0, center))


def test_rigid_particle_in_rest_fluid_stays_at_rest():
    s = oracle.Sim(_wl(24, 20, [_rigid_particle([11.0, 9.7])]))
    X0 = s.bodies[0].X.copy()
    s.step(30)
    assert np.max(np.abs(s.bodies[0].X - X0)) < 1e-13
    assert np.max(np.abs(s.bodies[0].U)) < 1e-14


def test_soft_particle_in_rest_fluid_stays_at_rest():
    xy = geometry.place(geometry.circle(3.0, 24), 0.0, [11.0, 9.7])
    b = configs.Body(configs.PARTICLE_SOFT, xy, ks=0.02, kb=0.002)
    s = oracle.Sim(_wl(24, 20, [b]))
    s.step(30)
    assert np.max(np.abs(s.bodies[0].X - xy)) < 1e-13


@pytest.mark.slow
def test_rigid_particle_carried_by_uniform_flow():
    nx = ny = 32
    u0 = np.zeros((2, ny, nx))
    u0[0] = 0.01
    s = oracle.Sim(_wl(nx, ny, [_rigid_particle([16.0, 16.0])], periodic_y=1, u0=u0))
    for _ in range(1500):
        s.step(1)
    U = s.bodies[0].U
    um = (s.rho * s.ux).sum() / s.rho.sum()
    assert abs(U[0] - um) < 0.02 * um
    assert abs(U[1]) < 1e-3 * um
    assert 0.8 * 0.01 < um <= 0.01 + 1e-12


def _max_coupling_force(s, steps):
    out = []
    for _ in range(steps):
        s.step(1)
        F = float(np.abs(s.marker_force[1]).max())
        out.append(F)
        if not np.isfinite(F):
            break
    return np.array(out)


def test_literal_verlet_velocity_coupling_grows_next_to_a_wall():
    """Evidence for the imposed soft-vertex velocity: with the second-order
    velocity of Eq. verletVel, U = 3/2 X^{n+1} - 2 X^n + 1/2 X^{n-1}, the
    weak-coupling force of the soft particle released at y_cr/2 from the wall
    (the gradient-window fixture) grows geometrically, about x1.2 per step,
    while the displacement velocity X^{n+1} - X^n keeps it at its initial size.
    Bounded: 56 steps, stops at the first non-finite force."""
    wl = configs.adjoint_channel()
    lit = oracle.Sim(wl)
    lit.soft_velocity = "verlet"
    F_lit = _max_coupling_force(lit, 56)
    F_disp = _max_coupling_force(oracle.Sim(wl), 56)
    assert np.all(np.isfinite(F_disp)) and F_disp.max() < 2.0 * F_disp[:5].max()
    assert F_lit[-1] > 100.0 * F_lit[:10].max()
    rate = (F_lit[50] / F_lit[30]) ** (1 / 20)
    assert rate > 1.1
