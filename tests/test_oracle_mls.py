"""Pins of the oracle's moving-least-squares transfer (Sec. 2.2, Immersed
Boundary Treatment; Sec. 2.3, nine nodes in a square of side 2.6 dx).

Each pin is fixed by the mathematics, not by the oracle's own formula:
  * a linear basis reproduces constants and linear functions exactly, for
    any weight and next to walls;
  * with the Roma kernel as the weight and all nine nodes inside the fluid,
    the moment matrix is diagonal, so the shape functions are the kernel;
  * the value at X equals a weighted least-squares fit solved by
    numpy.linalg.lstsq on the same nodes and weights (brute force);
  * the derivatives equal central differences of the shape functions;
  * spreading is the transpose of interpolation, so it conserves the total
    force and torque.
"""
import numpy as np
import pytest

from oracle import ib

WEIGHTS = [ib.Transfer("mls", "cubic", 1.3), ib.Transfer("mls", "gauss", 1.3),
           ib.Transfer("mls", "roma"), ib.Transfer("mls", "cubic", 1.05),
           ib.Transfer("mls", "gauss", 1.5)]


def points(n, nx, ny, seed, y_lo=0.0, y_hi=None):
    rng = np.random.default_rng(seed)
    y_hi = ny - 1.0 if y_hi is None else y_hi
    return np.stack([rng.uniform(0.0, nx, n), rng.uniform(y_lo, y_hi, n)], axis=1)


def node_xy(ix, iy, XY, nx):
    """Unwrapped node coordinates of each point's stencil, (M, 3, 3) each."""
    cx = np.floor(XY[:, 0] + 0.5)
    cy = np.floor(XY[:, 1] + 0.5)
    x = cx[:, None, None] + np.arange(-1, 2)[None, :, None] + 0 * np.arange(3)[None, None, :]
    y = cy[:, None, None] + np.arange(-1, 2)[None, None, :] + 0 * np.arange(3)[None, :, None]
    return x, y


@pytest.mark.parametrize("tr", WEIGHTS, ids=lambda t: f"{t.weight}-{t.h}")
@pytest.mark.parametrize("periodic_y", [False, True])
def test_reproduces_linear_functions(tr, periodic_y):
    nx, ny = 24, 12
    XY = points(400, nx, ny, 3, y_lo=0.0, y_hi=ny - 1.0)
    ix, iy, ph, dX, dY = ib.mls_shape(XY, nx, ny, periodic_y, tr)
    x, y = node_xy(ix, iy, XY, nx)
    assert np.abs(ph.sum(axis=(1, 2)) - 1.0).max() < 1e-13
    assert np.abs((ph * x).sum(axis=(1, 2)) - XY[:, 0]).max() < 1e-12
    assert np.abs((ph * y).sum(axis=(1, 2)) - XY[:, 1]).max() < 1e-12
    # derivatives of the reproduced fields: d(1) = 0, d(x)/dX = 1, d(y)/dY = 1
    assert np.abs(dX.sum(axis=(1, 2))).max() < 1e-12
    assert np.abs(dY.sum(axis=(1, 2))).max() < 1e-12
    assert np.abs((dX * x).sum(axis=(1, 2)) - 1.0).max() < 1e-12
    assert np.abs((dY * y).sum(axis=(1, 2)) - 1.0).max() < 1e-12
    assert np.abs((dX * y).sum(axis=(1, 2))).max() < 1e-12
    assert np.abs((dY * x).sum(axis=(1, 2))).max() < 1e-12


def test_linear_field_interpolated_exactly_through_public_calls():
    nx, ny = 20, 10
    tr = ib.Transfer("mls", "cubic", 1.3)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    field = 0.1 - 0.03 * xx + 0.07 * yy
    XY = points(200, nx - 3, ny, 5)          # stencils inside columns 0..nx-1: no periodic seam
    XY[:, 0] += 1.0
    want = 0.1 - 0.03 * XY[:, 0] + 0.07 * XY[:, 1]
    assert np.abs(ib.interpolate(field, XY, False, tr) - want).max() < 1e-12
    gx, gy = ib.interpolate_gradient(field, XY, False, tr)
    assert np.abs(gx + 0.03).max() < 1e-12 and np.abs(gy - 0.07).max() < 1e-12


def test_roma_weight_in_the_interior_is_the_roma_kernel():
    nx, ny = 30, 14
    XY = points(500, nx, ny, 7, y_lo=1.5, y_hi=ny - 2.5)    # all nine nodes inside the fluid
    ix, iy, ph, dX, dY = ib.mls_shape(XY, nx, ny, False, ib.Transfer("mls", "roma"))
    _, _, ddx, ddy, _, _ = ib._weights(XY, nx, ny, False)
    wx, wy = ib.phi(ddx), ib.phi(ddy)
    gx, gy = ib.dphi(ddx), ib.dphi(ddy)
    assert np.abs(ph - wx[:, :, None] * wy[:, None, :]).max() < 1e-14
    assert np.abs(dX + gx[:, :, None] * wy[:, None, :]).max() < 1e-13
    assert np.abs(dY + wx[:, :, None] * gy[:, None, :]).max() < 1e-13


def test_next_to_a_wall_the_fit_is_renormalised_not_truncated():
    nx, ny = 16, 8
    XY = np.array([[5.3, 0.2], [9.7, ny - 1.1]])
    f = np.ones((ny, nx))
    tr = ib.Transfer("mls", "roma")
    assert np.abs(ib.interpolate(f, XY, False, tr) - 1.0).max() < 1e-14
    assert np.all(ib.interpolate(f, XY, False) < 1.0 - 1e-3)    # the kernel loses the row beyond


@pytest.mark.parametrize("tr", WEIGHTS[:3], ids=lambda t: t.weight)
def test_value_equals_weighted_least_squares_fit(tr):
    nx, ny = 18, 9
    rng = np.random.default_rng(11)
    field = rng.normal(size=(ny, nx))
    XY = points(60, nx, ny, 13, y_lo=-0.25, y_hi=ny - 0.75)
    got = ib.interpolate(field, XY, False, tr)
    h = ib.support(tr)
    for k, (X, Y) in enumerate(XY):
        rows, vals, wts = [], [], []
        cx, cy = int(np.floor(X + 0.5)), int(np.floor(Y + 0.5))
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                xn, yn = cx + a, cy + b
                if yn < 0 or yn >= ny:
                    continue
                wx_, _ = ib.weight(np.array([xn - X]), tr)
                wy_, _ = ib.weight(np.array([yn - Y]), tr)
                rows.append((xn - X, yn - Y))
                vals.append(field[yn, xn % nx])
                wts.append(wx_[0] * wy_[0])
        rows, vals, wts = np.array(rows), np.array(vals), np.array(wts)
        inside = np.unique(rows[wts > 0, 1]).size
        basis = [np.ones(len(rows)), rows[:, 0]] + ([rows[:, 1]] if inside >= 2 else [])
        Pm = np.stack(basis, axis=1)
        sw = np.sqrt(wts)
        coef, *_ = np.linalg.lstsq(Pm * sw[:, None], vals * sw, rcond=None)
        assert abs(got[k] - coef[0]) < 1e-11, (k, X, Y)


@pytest.mark.parametrize("tr", WEIGHTS[:3], ids=lambda t: t.weight)
def test_derivatives_match_central_differences(tr):
    nx, ny = 18, 9
    XY = points(200, nx, ny, 17, y_lo=0.6, y_hi=ny - 1.6)
    # stay away from the stencil switch at half-integers (the FD step would cross it)
    frac = XY - np.floor(XY)
    keep = np.all(np.abs(frac - 0.5) > 1e-3, axis=1)
    XY = XY[keep]
    eps = 1e-6
    _, _, _, dX, dY = ib.mls_shape(XY, nx, ny, False, tr)
    for d, D in ((0, dX), (1, dY)):
        e = np.zeros(2)
        e[d] = eps
        _, _, pp, _, _ = ib.mls_shape(XY + e, nx, ny, False, tr)
        _, _, pm, _, _ = ib.mls_shape(XY - e, nx, ny, False, tr)
        fd = (pp - pm) / (2 * eps)
        assert np.abs(fd - D).max() < 2e-7


def test_spread_is_the_transpose_and_conserves_force_and_torque():
    nx, ny = 22, 11
    tr = ib.Transfer("mls", "gauss", 1.3)
    rng = np.random.default_rng(19)
    XY = points(80, nx, ny, 23, y_lo=0.0, y_hi=ny - 1.0)
    F = rng.normal(size=(80, 2))
    E = ib.spread(F, XY, nx, ny, False, tr)
    u = rng.normal(size=(ny, nx))
    v = rng.normal(size=(ny, nx))
    lhs = (E[0] * u).sum() + (E[1] * v).sum()
    rhs = (F[:, 0] * ib.interpolate(u, XY, False, tr)).sum() + (F[:, 1] * ib.interpolate(v, XY, False, tr)).sum()
    assert abs(lhs - rhs) < 1e-11 * (1 + abs(lhs))
    assert np.abs(E.sum(axis=(1, 2)) - F.sum(axis=0)).max() < 1e-12
    # torque about the origin, x unwrapped: keep the points off the periodic seam
    XY2 = XY.copy()
    XY2[:, 0] = 2.0 + XY2[:, 0] * (nx - 4.0) / nx
    E2 = ib.spread(F, XY2, nx, ny, False, tr)
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    tq_grid = (xx * E2[1] - yy * E2[0]).sum()
    tq = (XY2[:, 0] * F[:, 1] - XY2[:, 1] * F[:, 0]).sum()
    assert abs(tq_grid - tq) < 1e-10


def test_degenerate_stencil_drops_the_y_term():
    # beyond the halfway wall by more than h - 1: only row 0 is inside the support
    nx, ny = 12, 6
    tr = ib.Transfer("mls", "cubic", 1.3)
    XY = np.array([[4.2, -0.4]])
    ix, iy, ph, dX, dY = ib.mls_shape(XY, nx, ny, False, tr)
    assert np.all(np.isfinite(ph)) and abs(ph.sum() - 1.0) < 1e-14
    f = np.tile(np.arange(ny, dtype=float)[:, None], (1, nx))      # f = y
    assert abs(ib.interpolate(f, XY, False, tr)[0] - 0.0) < 1e-14  # constant along y: row 0's value
