"""Pins of the oracle's Zou-He velocity walls (the paper's wall condition,
Sec. 2.1) on the node rows 0 and ny - 1: the defining conditions of the
reconstruction, Couette flow (an exact linear steady state of the lattice
equation) and forced Poiseuille flow (steady state: the parabola with channel
height ny - 1, exact only if the half-force velocity at a wall node is the
wall velocity, the reading of the wall forcing)."""
import numpy as np
import pytest

from oracle import lattice as L
from oracle import sim as osim
from workloads import configs


def _fields(nx, ny, ux):
    u = np.tile(np.asarray(ux, dtype=np.float64)[:, None], (1, nx))
    return np.ones((ny, nx)), u, np.zeros((ny, nx))


def test_reconstruction_sets_density_and_wall_velocity():
    rng = np.random.default_rng(3)
    nx, ny = 7, 6
    f = L.W[:, None, None] * (1.0 + 0.05 * rng.standard_normal((9, ny, nx)))
    fs = L.stream(f, False, True)
    assert np.isnan(fs[[2, 5, 6], 0]).all() and np.isnan(fs[[4, 7, 8], ny - 1]).all()
    fx = 1e-3 * rng.standard_normal((ny, nx))
    fy = 1e-3 * rng.standard_normal((ny, nx))
    u_lo, u_hi = 0.013, -0.021
    g = L.zou_he(fs, fx, fy, u_lo, u_hi)
    known = ~np.isnan(fs)
    assert np.array_equal(g[known], fs[known])                  # known populations untouched
    for y, uw in ((0, u_lo), (ny - 1, u_hi)):
        rho = g[:, y].sum(axis=0)
        jx = (L.E[:, 0, None] * g[:, y]).sum(axis=0)
        jy = (L.E[:, 1, None] * g[:, y]).sum(axis=0)
        assert np.allclose((jx + 0.5 * fx[y]) / rho, uw, atol=1e-15, rtol=0)
        assert np.allclose((jy + 0.5 * fy[y]) / rho, 0.0, atol=1e-15, rtol=0)


def _run(nx, ny, tau, u_hi, g, steps, ux0):
    rho, ux, uy = _fields(nx, ny, ux0)
    f = L.equilibrium(rho, ux, uy)
    fx, fy = np.full((ny, nx), g), np.zeros((ny, nx))
    for _ in range(steps):
        f, rho, ux, uy = L.collide(L.zou_he(L.stream(f, False, True), fx, fy, 0.0, u_hi), fx, fy, tau)
    return rho, ux, uy


def test_couette_linear_profile_is_exact():
    ny, U = 12, 0.05
    y = np.arange(ny)
    rho, ux, uy = _run(4, ny, 0.8, U, 0.0, 300, U * y / (ny - 1))
    assert np.abs(ux - U * y[:, None] / (ny - 1)).max() < 1e-13
    assert np.abs(rho - 1).max() < 1e-13 and np.abs(uy).max() < 1e-14


def test_couette_from_rest_converges_to_the_line():
    ny, U = 10, 0.05
    y = np.arange(ny)
    _, ux, _ = _run(3, ny, 0.8, U, 0.0, 6000, np.zeros(ny))
    assert np.abs(ux - U * y[:, None] / (ny - 1)).max() < 1e-12


@pytest.mark.parametrize("tau,steps", [(0.8, 20000), (1.0, 10000)])
def test_forced_poiseuille_steady_state_is_the_parabola(tau, steps):
    ny, g = 11, 1e-6
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny)
    exact = g / (2.0 * nu) * y * (ny - 1 - y)
    _, ux, _ = _run(2, ny, tau, 0.0, g, steps, exact)
    assert np.abs(ux - exact[:, None]).max() / exact.max() < 1e-9


def test_sim_uses_wall_positions_for_bonds():
    # a particle centroid 0.4 above the lower wall: eligible for a bond with
    # y_cr = 0.5 only if the wall is on row 0 (zou-he), not at -1/2
    from oracle import adhesion
    assert adhesion.nearer_wall(0.4, 20, (0.0, 19.0)) == (0, pytest.approx(0.4))
    assert adhesion.nearer_wall(0.4, 20) == (0, pytest.approx(0.9))
    assert adhesion.bond_length((3.0, 0.4), 3.0, 0, 10, 20, (0.0, 19.0)) == pytest.approx(0.4)
    wl = configs.Workload("w", 8, 6, walls="zou-he", u_wall=(0.0, 0.01))
    s = osim.Sim(wl)
    s.step(2)
    assert s.y_walls == (0.0, 5.0) and s.wet_walls
