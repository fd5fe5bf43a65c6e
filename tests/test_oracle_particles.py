"""Pins of the oracle's probe loads and particle integrators (Sec. 2.2-2.3)."""
import numpy as np
import pytest

import oracle
from oracle import ib, lattice, membrane, particles
from workloads import configs, geometry


def test_probe_loads_in_linear_fields_closed_form():
    """rho = 1 + a x + b y, u = gamma y, v = kappa x: the kernel interpolant and
    its gradient are exact for linear fields, so each element load is known:
    F^p = -cs^2 (a q_x + b q_y) n l, F^tau = rho0 nu (gamma + kappa) (n_y, n_x) l."""
    nx, ny = 64, 40
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, gam, kap = 2e-4, -3e-4, 1e-3, -4e-4
    rho = 1 + a * x + b * y
    u, v = gam * y, kap * x
    xy = geometry.place(geometry.circle(5.0, 30), 0.2, [30.0, 18.0])
    nu = 0.1
    F = particles.hydro_element_forces(xy, rho, u, v, nu, periodic_y=False)
    length, _, n = membrane.elements(xy)
    q = membrane.centroids(xy) + 1.2 * n
    p = (a * q[:, 0] + b * q[:, 1]) / 3
    ex = np.stack([-p * n[:, 0] + nu * (gam + kap) * n[:, 1],
                   -p * n[:, 1] + nu * (gam + kap) * n[:, 0]], 1) * length[:, None]
    assert np.max(np.abs(F - ex)) < 1e-15


def test_probe_clamped_inside_fluid():
    xy = geometry.place(geometry.circle(3.0, 24), 0.0, [10.0, 2.0])
    q = particles.probe_points(xy, 20, periodic_y=False)
    assert q[:, 1].min() >= 0.5 and q[:, 1].max() <= 18.5
    assert (particles.probe_points(xy, 20, periodic_y=True)[:, 1] < 0.5).any()


def test_bdf2_constant_rate_and_start():
    # constant acceleration a: exact BDF2 recursion from rest
    a = 0.01
    v_prev, v = 0.0, 0.0
    v1 = particles.bdf2(v, v_prev, a, first=True)
    assert v1 == a
    v2 = particles.bdf2(v1, v, a, first=False)
    assert abs(v2 - (2 / 3) * (2 * a + a)) < 1e-18


def test_marker_weights_sum_to_perimeter():
    xy = geometry.rbc_contour(20.0, 100)
    length, _, _ = membrane.elements(xy)
    assert abs(particles.marker_weights(xy).sum() - length.sum()) < 1e-12


# ---------------------------------------------------------------------------
# Pins of the rigid inertia, the Verlet step and the weak-coupling gain.

def _polygon_second_moment(xy):
    """Exact polar second moment of area of a simple polygon about its area
    centroid (Green's theorem over the edges), and its area."""
    x, y = xy[:, 0], xy[:, 1]
    x1, y1 = np.roll(x, -1), np.roll(y, -1)
    c = x * y1 - x1 * y
    A = c.sum() / 2
    cx = ((x + x1) * c).sum() / (6 * A)
    cy = ((y + y1) * c).sum() / (6 * A)
    Ixx = ((y * y + y * y1 + y1 * y1) * c).sum() / 12
    Iyy = ((x * x + x * x1 + x1 * x1) * c).sum() / 12
    return Ixx + Iyy - A * (cx * cx + cy * cy), A


@pytest.mark.parametrize("n, r", [(40, 3.2), (216, 33.3)])
def test_rigid_inertia_is_second_moment_of_the_disc(n, r):
    """Eq. angularVelRig needs I: the particle is a disc of density
    rho_P = 1.1 rho0 (Sec. 3), so I = rho_P times the polar second moment of
    its area, computed here exactly for the polygon (differs from the disc's
    m r^2 / 2 by O(1/n^2))."""
    xy = geometry.place(geometry.circle(r, n), 0.3, [40.0, 20.0])
    b = oracle.sim.BodyState(oracle.sim.PARTICLE_RIGID, xy, 0, 0, 1, 1 / 3, 1.1, 0, 0)
    J, A = _polygon_second_moment(xy)
    assert abs(b.mass - 1.1 * A) < 1e-12 * b.mass
    assert abs(b.inertia / (1.1 * J) - 1.0) < 0.01


def _bonded_particle_sim(kind, xy, sigma, lig_elem):
    """Particle at rest next to the lower wall in fluid at rest, one frozen bond
    on element lig_elem to the receptor below its centroid."""
    nx, ny = 48, 24
    wl = configs.Workload("pin", nx, ny, 1.0, bodies=[
        configs.Body(kind, xy, ks=0.02, kb=1e-3, sigma=sigma, ligand_stride=1)],
        receptors=configs.uniform_receptors(nx),
        adhesion=configs.Adhesion(y_cr=2.0, y_eq=0.25, kf0_dt=0.0, kr0_dt=0.0,
                                  sigma_ts_frac=0.5, kbt=1.0, freeze_topology=1))
    s = oracle.Sim(wl)
    c = 0.5 * (xy[lig_elem] + xy[(lig_elem + 1) % len(xy)])
    s.l2r[lig_elem] = int(round(c[0]))          # receptor x = 0..nx-1 on the lower wall
    return s, c


def _bond_force(xy, e, sigma, y_eq):
    """sigma (y_l - y_eq) n_l of Eq. adhFor for a receptor on the lower wall
    (y = -1/2) straight below the element centroid."""
    d = xy[(e + 1) % len(xy)] - xy[e]
    n = np.array([d[1], -d[0]]) / np.hypot(*d)
    c = 0.5 * (xy[e] + xy[(e + 1) % len(xy)])
    yl = np.hypot(c[0] - round(c[0]), c[1] + 0.5)
    return sigma * (yl - y_eq) * n, c


def test_rigid_first_step_follows_force_and_moment():
    """One step of a rigid particle at rest in fluid at rest whose only load is
    one bond spring: U^1 = F/m and Omega^1 = M/I (forward Euler start of Eqs.
    linearVelRig, angularVelRig); the pre-forcing fluid at rest carries no
    probe load.  The polygon is a 40-gon with one vertex moved so that the
    bonded element's normal misses the centre and the spring exerts a moment."""
    xy = geometry.place(geometry.circle(3.2, 40), 0.0, [24.0, 3.0])
    xy[31] += np.array([0.35, -0.15])           # tilt element 30 (faces the lower wall)
    sigma, e = 5e-3, 30
    s, c = _bonded_particle_sim(oracle.sim.PARTICLE_RIGID, xy, sigma, e)
    F, c = _bond_force(xy, e, sigma, 0.25)
    Xc = xy.mean(axis=0)
    M = (c[0] - Xc[0]) * F[1] - (c[1] - Xc[1]) * F[0]
    assert abs(M) > 0.05 * np.hypot(*F)         # a real moment arm
    J, A = _polygon_second_moment(xy)
    s.step(1)
    b = s.bodies[0]
    assert np.max(np.abs(b.U - F / (1.1 * A))) < 1e-12 * np.hypot(*F) / A
    assert abs(b.Om / (M / (1.1 * J)) - 1.0) < 0.02


def test_soft_first_step_moves_vertices_by_half_force_over_mass():
    """Eq. verletPos with dt = 1 from rest: X^1 = X^0 + U_0 + F/(2 m_v), U_0 = 0 in
    fluid at rest, m_v = 1.1 rho0 A_0 / n_v (mass spread evenly over the
    vertices).  The stress-free particle's only load is one bond spring, half
    on each vertex of its element (Sec. 2.2)."""
    nv = 40
    xy = geometry.place(geometry.circle(3.2, nv), 0.0, [24.0, 3.0])
    sigma, e = 5e-3, 30
    s, _ = _bonded_particle_sim(oracle.sim.PARTICLE_SOFT, xy, sigma, e)
    F, _ = _bond_force(xy, e, sigma, 0.25)
    _, A = _polygon_second_moment(xy)
    mv = 1.1 * A / nv
    s.step(1)
    dX = s.bodies[0].X - xy
    expected = np.zeros_like(xy)
    expected[e] = expected[(e + 1) % nv] = 0.5 * F / (2 * mv)
    assert np.max(np.abs(expected)) > 1e-4
    # X + dX rounds at |X| ~ 24
    assert np.max(np.abs(dX - expected)) < 1e-13


def test_direct_forcing_gain_gives_the_imposed_velocity():
    """The weak coupling's gain 2 rho0 is what makes one LB step with the half-force
    velocity of Sec. 2.2 (rho u = sum f e + F/2) reproduce the imposed marker
    velocity: markers on every node of a periodic box (ds = 1, the kernel's
    partition of unity gives F(x) = F_k everywhere) and fluid at rest give
    u = U exactly after the step."""
    nx, ny = 6, 5
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    XY = np.stack([xx.ravel(), yy.ravel()], axis=1)
    U = np.tile([[0.013, -0.021]], (len(XY), 1))
    F = particles.direct_forcing(U, np.zeros_like(U), np.ones(len(XY)))
    FE = ib.spread(F, XY, nx, ny, periodic_y=True)
    f0 = lattice.equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    _, rho, ux, uy = lattice.collide(f0, FE[0], FE[1], 1.0)
    assert np.max(np.abs(ux - 0.013)) < 1e-16 and np.max(np.abs(uy + 0.021)) < 1e-16
