"""Pins of the oracle's lattice Boltzmann part (Sec. 2.1-2.2 of the paper).

Each check compares against something other than the oracle itself:
closed-form moments of the D2Q9 equilibrium and of Guo's source, the exact
steady channel profile of BGK + halfway bounce-back + Guo forcing, exact
conservation laws, the decay rate of a shear wave, and a loop-only
push-streaming implementation on tiny lattices.
"""
import numpy as np
import pytest

from oracle import lattice
from workloads import configs

E, W, OPP = lattice.E, lattice.W, lattice.OPP


def test_velocity_set_matches_listing():
    # Eq. (GaussHermite) evaluated must give the standard D2Q9 set
    ref = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    assert (E == ref).all()
    assert list(OPP) == [0, 3, 4, 1, 2, 7, 8, 5, 6]
    assert abs(W.sum() - 1.0) < 1e-15
    # isotropy: sum w e_a e_b = cs^2 delta_ab, 4th-order isotropic
    T2 = np.einsum("i,ia,ib->ab", W, E, E)
    assert np.allclose(T2, np.eye(2) / 3.0, atol=1e-15)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", W, E, E, E, E)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(T4, iso, atol=1e-15)


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.1 * rng.standard_normal((3, 4))
    ux, uy = 0.05 * rng.standard_normal((2, 3, 4))
    feq = lattice.equilibrium(rho, ux, uy)
    assert np.allclose(feq.sum(0), rho, atol=1e-14)
    jx, jy = lattice.momentum(feq)
    assert np.allclose(jx, rho * ux, atol=1e-14)
    assert np.allclose(jy, rho * uy, atol=1e-14)
    # second moment: rho cs^2 I + rho u u
    Pxx = np.einsum("i,iyx->yx", E[:, 0] * E[:, 0] * 1.0, feq)
    Pxy = np.einsum("i,iyx->yx", E[:, 0] * E[:, 1] * 1.0, feq)
    Pyy = np.einsum("i,iyx->yx", E[:, 1] * E[:, 1] * 1.0, feq)
    assert np.allclose(Pxx, rho / 3 + rho * ux * ux, atol=1e-14)
    assert np.allclose(Pxy, rho * ux * uy, atol=1e-14)
    assert np.allclose(Pyy, rho / 3 + rho * uy * uy, atol=1e-14)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_guo_source_moments(tau):
    # Guo's term: zeroth moment 0, first (1 - 1/2tau) F, second (1 - 1/2tau)(uF + Fu)
    rng = np.random.default_rng(1)
    ux, uy, fx, fy = 0.05 * rng.standard_normal((4, 5))
    S = lattice.guo_source(ux, uy, fx, fy, tau)
    pre = 1 - 1 / (2 * tau)
    assert np.allclose(S.sum(0), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,i...->...", E[:, 0] * 1.0, S), pre * fx, atol=1e-16)
    assert np.allclose(np.einsum("i,i...->...", E[:, 1] * 1.0, S), pre * fy, atol=1e-16)
    Sxx = np.einsum("i,i...->...", E[:, 0] * E[:, 0] * 1.0, S)
    Sxy = np.einsum("i,i...->...", E[:, 0] * E[:, 1] * 1.0, S)
    assert np.allclose(Sxx, pre * 2 * ux * fx, atol=1e-16)
    assert np.allclose(Sxy, pre * (ux * fy + uy * fx), atol=1e-16)


def _run_channel(nx, ny, tau, g, steps, u0=None):
    rho0 = np.ones((ny, nx))
    if u0 is None:
        u0 = np.zeros((2, ny, nx))
    f = lattice.equilibrium(rho0, u0[0], u0[1])
    fx = np.full((ny, nx), g)
    fy = np.zeros((ny, nx))
    for _ in range(steps):
        f, rho, ux, uy = lattice.lb_step(f, fx, fy, tau)
    return f, rho, ux, uy


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0, 0.5 + np.sqrt(3.0 / 16.0), 1.5])
def test_poiseuille_closed_form(tau):
    # steady u(y) = g/(2 nu) [(y + 1/2)(ny - 1/2 - y) + (16 L - 3)/12], L = (tau - 1/2)^2
    nx, ny, g = 4, 10, 1e-5
    prof = configs.poiseuille_profile(g, ny, tau)
    u0 = np.zeros((2, ny, nx))
    u0[0] = 0.9 * prof[:, None]
    f, rho, ux, uy = _run_channel(nx, ny, tau, g, 9000, u0)
    nu = (tau - 0.5) / 3
    scale = g / (2 * nu)
    assert np.max(np.abs(ux - prof[:, None])) < 1e-9 * scale
    assert np.max(np.abs(uy)) < 1e-13
    # the slip term matters: plain parabola is off by g/(24 nu) at tau = 1
    if tau == 1.0:
        plain = scale * (np.arange(ny) + 0.5) * (ny - 0.5 - np.arange(ny))
        assert np.max(np.abs(ux - plain[:, None])) > 0.9 * g / (24 * nu)


def test_mass_conserved_with_walls_and_force():
    rng = np.random.default_rng(2)
    nx, ny = 12, 9
    f = lattice.equilibrium(1 + 0.01 * rng.standard_normal((ny, nx)),
                            *(0.02 * rng.standard_normal((2, ny, nx))))
    m0 = f.sum()
    for _ in range(50):
        fx, fy = 1e-3 * rng.standard_normal((2, ny, nx))
        f, rho, ux, uy = lattice.lb_step(f, fx, fy, 0.8)
    assert abs(f.sum() - m0) < 1e-11


def test_momentum_budget_periodic_box():
    # periodic in x and y: total physical momentum changes by (F^n + F^{n+1})/2 summed
    rng = np.random.default_rng(3)
    nx, ny, tau = 10, 8, 0.9
    f = lattice.equilibrium(np.ones((ny, nx)), *(0.01 * rng.standard_normal((2, ny, nx))))
    Fprev = np.zeros((2, ny, nx))
    # physical momentum at step 0 with zero force
    f, rho, ux, uy = lattice.lb_step(f, Fprev[0], Fprev[1], tau, periodic_y=True)
    P = np.array([(rho * ux).sum(), (rho * uy).sum()])
    for _ in range(20):
        F = 1e-4 * rng.standard_normal((2, ny, nx))
        f, rho, ux, uy = lattice.lb_step(f, F[0], F[1], tau, periodic_y=True)
        Pn = np.array([(rho * ux).sum(), (rho * uy).sum()])
        expect = P + 0.5 * (Fprev.sum(axis=(1, 2)) + F.sum(axis=(1, 2)))
        assert np.allclose(Pn, expect, atol=1e-14)
        P, Fprev = Pn, F


def test_rest_state_is_fixed_point_and_uniform_flow_stays_uniform():
    nx, ny = 7, 5
    f = lattice.equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    z = np.zeros((ny, nx))
    f1, rho, ux, uy = lattice.lb_step(f, z, z, 1.0)
    assert np.max(np.abs(f1 - f)) < 1e-15  # rest state fixed up to the rounding of sum w_i
    u0 = 0.03
    f = lattice.equilibrium(np.ones((ny, nx)), np.full((ny, nx), u0), np.full((ny, nx), -0.01))
    for _ in range(10):
        f, rho, ux, uy = lattice.lb_step(f, z, z, 0.7, periodic_y=True)
    assert np.allclose(ux, u0, atol=1e-15) and np.allclose(uy, -0.01, atol=1e-15)


def test_shear_wave_decay():
    # u_x = U0 sin(k y) decays as exp(-nu k^2 t) up to O(k^2) lattice corrections
    nx, ny, tau, U0 = 4, 64, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / ny
    y = np.arange(ny)
    u0 = np.zeros((2, ny, nx))
    u0[0] = U0 * np.sin(k * y)[:, None]
    f = lattice.equilibrium(np.ones((ny, nx)), u0[0], u0[1])
    z = np.zeros((ny, nx))
    T = 400
    for _ in range(T):
        f, rho, ux, uy = lattice.lb_step(f, z, z, tau, periodic_y=True)
    amp = 2 * np.mean(ux[:, 0] * np.sin(k * y))
    expect = U0 * np.exp(-nu * k * k * T)
    assert abs(amp / expect - 1) < 5e-3


def _push_loop(fpost, tau, fx, fy, periodic_y):
    """Loop-only push streaming + collision, written without array shifts."""
    _, ny, nx = fpost.shape
    ex = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    w = [4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]
    opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
    fpre = np.zeros_like(fpost)
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                xd = (x + ex[i]) % nx
                yd = y + ey[i]
                if periodic_y:
                    fpre[i, yd % ny, xd] = fpost[i, y, x]
                elif 0 <= yd < ny:
                    fpre[i, yd, xd] = fpost[i, y, x]
                else:  # reflected back into the node it left, opposite direction
                    fpre[opp[i], y, x] = fpost[i, y, x]
    out = np.zeros_like(fpost)
    for y in range(ny):
        for x in range(nx):
            rho = sum(fpre[i, y, x] for i in range(9))
            ux = (sum(fpre[i, y, x] * ex[i] for i in range(9)) + 0.5 * fx[y, x]) / rho
            uy = (sum(fpre[i, y, x] * ey[i] for i in range(9)) + 0.5 * fy[y, x]) / rho
            for i in range(9):
                eu = ex[i] * ux + ey[i] * uy
                feq = w[i] * rho * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy))
                src = (1 - 0.5 / tau) * w[i] * (
                    (3 * (ex[i] - ux) + 9 * eu * ex[i]) * fx[y, x]
                    + (3 * (ey[i] - uy) + 9 * eu * ey[i]) * fy[y, x])
                out[i, y, x] = fpre[i, y, x] - (fpre[i, y, x] - feq) / tau + src
    return out


@pytest.mark.parametrize("shape,periodic_y", [((5, 6), False), ((4, 3), True), ((1, 1), False),
                                              ((2, 3), False)])
def test_bruteforce_push_matches(shape, periodic_y):
    ny, nx = shape
    rng = np.random.default_rng(4)
    f = lattice.equilibrium(1 + 0.05 * rng.random((ny, nx)), *(0.05 * rng.standard_normal((2, ny, nx))))
    f += 0.001 * rng.standard_normal(f.shape)
    fx, fy = 1e-3 * rng.standard_normal((2, ny, nx))
    a, *_ = lattice.lb_step(f, fx, fy, 0.85, periodic_y)
    b = _push_loop(f, 0.85, fx, fy, periodic_y)
    assert np.max(np.abs(a - b)) < 1e-14
