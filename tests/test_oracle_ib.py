"""Pins of the oracle's immersed-boundary transfer (Sec. 2.2-2.3 of the paper).

Closed-form moments of the Roma kernel, exact reproduction of linear
fields, the exact quadratic correction, the spread/interpolate adjoint
identity, and whole-lattice spreading without a stencil (brute force).
"""
import numpy as np
import pytest

from oracle import ib


def test_kernel_closed_form_values():
    assert ib.phi(np.array([0.0]))[0] == pytest.approx(2 / 3, abs=1e-16)
    assert ib.phi(np.array([1.0]))[0] == pytest.approx(1 / 6, abs=1e-16)
    assert ib.phi(np.array([0.5]))[0] == pytest.approx(0.5, abs=1e-16)
    assert ib.phi(np.array([1.5]))[0] == pytest.approx(0.0, abs=1e-16)
    assert ib.phi(np.array([1.6]))[0] == 0.0


@pytest.mark.parametrize("X", np.linspace(-3.0, 3.0, 37) + 0.0123)
def test_kernel_moments(X):
    j = np.arange(-6, 7)
    r = j - X
    w = ib.phi(r)
    assert abs(w.sum() - 1) < 1e-15                 # partition of unity
    assert abs((w * r).sum()) < 1e-15               # first moment
    assert abs((w * w).sum() - 0.5) < 1e-15         # sum phi^2 = 1/2
    m2 = (w * r * r).sum()
    assert 0.25 - 1e-15 <= m2 <= 1 / 3 + 1e-15
    # derivative: sum phi' = 0, sum phi' r = -1 (derivative of the moment identities)
    d = ib.dphi(r)
    assert abs(d.sum()) < 1e-14
    assert abs((d * r).sum() + 1) < 1e-14


def test_second_moment_extremes():
    for X, m in [(0.0, 1 / 3), (0.5, 0.25)]:
        j = np.arange(-4, 5)
        w = ib.phi(j - X)
        assert abs((w * (j - X) ** 2).sum() - m) < 1e-15


def test_dphi_matches_finite_difference():
    r = np.linspace(-1.6, 1.6, 161) + 1e-3
    h = 1e-6
    fd = (ib.phi(r + h) - ib.phi(r - h)) / (2 * h)
    assert np.max(np.abs(fd - ib.dphi(r))) < 1e-7


def test_interpolation_reproduces_linear_and_quadratic():
    nx, ny = 16, 12
    rng = np.random.default_rng(0)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    XY = np.stack([rng.uniform(0, nx), rng.uniform(2, ny - 3)] * 1)[None, :]
    XY = np.concatenate([XY, np.stack([rng.uniform(0, nx, 20), rng.uniform(2, ny - 3, 20)], 1)])
    lin = 0.3 + 0.7 * y
    assert np.allclose(ib.interpolate(lin, XY), 0.3 + 0.7 * XY[:, 1], atol=1e-14)
    quad = 2.0 * (y - 3.0) ** 2
    # U = u(Y) + u''/2 * m2(frac Y)
    Y = XY[:, 1]
    jj = np.floor(Y + 0.5)[:, None] + np.arange(-1, 2)[None, :]
    m2 = (ib.phi(jj - Y[:, None]) * (jj - Y[:, None]) ** 2).sum(1)
    assert np.allclose(ib.interpolate(quad, XY), 2.0 * (Y - 3) ** 2 + 2.0 * m2, atol=1e-13)
    # gradient of the interpolant of a linear field is exact
    gx, gy = ib.interpolate_gradient(0.3 + 0.5 * y - 0.2 * ((x - 0.0)), XY)
    # x is periodic, so keep markers away from the seam
    sel = (XY[:, 0] > 2) & (XY[:, 0] < nx - 3)
    assert np.allclose(gy[sel], 0.5, atol=1e-13) and np.allclose(gx[sel], -0.2, atol=1e-13)


def test_spread_interp_adjoint():
    nx, ny = 20, 14
    rng = np.random.default_rng(1)
    XY = np.stack([rng.uniform(-5, nx + 5, 30), rng.uniform(1.5, ny - 2.5, 30)], 1)
    F = rng.standard_normal((30, 2))
    u = rng.standard_normal((2, ny, nx))
    S = ib.spread(F, XY, nx, ny)
    lhs = (S * u).sum()
    rhs = (F[:, 0] * ib.interpolate(u[0], XY)).sum() + (F[:, 1] * ib.interpolate(u[1], XY)).sum()
    assert abs(lhs - rhs) < 1e-12
    # spreading conserves total force away from walls
    assert np.allclose(S.sum(axis=(1, 2)), F.sum(0), atol=1e-13)


@pytest.mark.parametrize("nx,ny,periodic_y", [(6, 5, False), (5, 4, True), (3, 6, False)])
def test_spread_bruteforce_whole_lattice(nx, ny, periodic_y):
    """Kernel evaluated at every node with minimum-image distances, no stencil."""
    rng = np.random.default_rng(2)
    M = 7
    XY = np.stack([rng.uniform(-10, 10, M), rng.uniform(-0.4, ny - 0.6, M)], 1)
    F = rng.standard_normal((M, 2))
    ref = np.zeros((2, ny, nx))
    for k in range(M):
        for yy in range(ny):
            for xx in range(nx):
                # all periodic images within reach of the kernel support
                for sx in range(-4, 5):
                    dx = xx + sx * nx - XY[k, 0]
                    wy_total = 0.0
                    if periodic_y:
                        for sy in range(-4, 5):
                            wy_total += ib.phi(np.array([yy + sy * ny - XY[k, 1]]))[0]
                    else:
                        wy_total = ib.phi(np.array([yy - XY[k, 1]]))[0]
                    w = ib.phi(np.array([dx]))[0] * wy_total
                    ref[:, yy, xx] += F[k] * w
    got = ib.spread(F, XY, nx, ny, periodic_y)
    if nx >= 3 and (not periodic_y or ny >= 3):
        assert np.max(np.abs(got - ref)) < 1e-14
