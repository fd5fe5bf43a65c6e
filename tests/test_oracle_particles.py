"""Pins of the oracle's probe loads and particle integrators (Sec. 2.2-2.3)."""
import numpy as np

from oracle import membrane, particles
from workloads import geometry


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
