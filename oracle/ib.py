"""Immersed-boundary transfer between the Lagrangian chain and the lattice (oracle).

Sec. 2.2 (Immersed Boundary Treatment) and Sec. 2.3 (Blood Cells Motion):
every Lagrangian point exchanges data with the nine lattice nodes around
it.  The paper names a moving-least-squares reconstruction; the reading
used here is the 3-point kernel of Roma, Peskin and Berger on the 3x3
nearest nodes.  With a linear basis and this kernel as the MLS weight the
moment matrix is diagonal (the kernel reproduces constants and linear
functions exactly), so the MLS shape functions reduce to the kernel
itself.

  phi(r) = (1 + sqrt(1 - 3 r^2)) / 3                 |r| <= 1/2
         = (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6   1/2 <= |r| <= 3/2
         = 0                                         otherwise
  delta(x - X) = phi(x - X) phi(y - Y)

Stencil: i in floor(X + 1/2) + {-1, 0, 1}, x periodic.  With walls, rows
outside 0..ny-1 are dropped (the fluid velocity beyond the wall is taken
as zero when interpolating; a spread share that falls there is dropped).

The general moving-least-squares reconstruction (Sec. 2.2, Immersed Boundary
Treatment; Sec. 2.3, nine nodes in a square of side 2.6 dx) is the
alternative `Transfer("mls", weight, h)`: a linear basis p = (1, x, y) fitted
by weighted least squares to the nodes of the same 3x3 stencil, with a
tensor-product weight W_j = w(x_j - X) w(y_j - Y) of support half-width h
(1.3 for the paper's square; 3/2, its own support, for the Roma weight).
The shape functions are phi_j(X) = p(X)^T A(X)^{-1} W_j(X) p(x_j) with the
moment matrix A = sum_j W_j p(x_j) p(x_j)^T; they reproduce constants and
linear functions exactly, so the transfer conserves force and torque.
Rows beyond a wall are not nodes of the fit (weight zero), so near a wall
the fit is one-sided and renormalised rather than truncated.  Readings: the
weight is a free choice (Roma, cubic spline, or Gaussian); a point whose
stencil has fewer than two rows inside the support drops the y term of the
basis (its fit is constant along y); spreading uses the same shape functions
(the transpose of the interpolation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def phi(r):
    """Roma 3-point kernel."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 0.5
    m2 = (a > 0.5) & (a <= 1.5)
    out[m1] = (1.0 + np.sqrt(1.0 - 3.0 * a[m1] ** 2)) / 3.0
    out[m2] = (5.0 - 3.0 * a[m2] - np.sqrt(np.maximum(0.0, 1.0 - 3.0 * (1.0 - a[m2]) ** 2))) / 6.0
    return out


def dphi(r):
    """Derivative of the Roma kernel with respect to its argument (C1 function)."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    s = np.sign(r)
    out = np.zeros_like(a)
    m1 = a <= 0.5
    m2 = (a > 0.5) & (a < 1.5)
    out[m1] = -r[m1] / np.sqrt(1.0 - 3.0 * r[m1] ** 2)
    b = 1.0 - a[m2]
    out[m2] = s[m2] * (-0.5 - b / (2.0 * np.sqrt(1.0 - 3.0 * b * b)))
    return out


def stencil(X: np.ndarray, n: int, periodic: bool):
    """Indices, offsets (node - X) and validity of the 3 nearest nodes per point.

    X: (M,) coordinates.  Returns idx (M, 3) wrapped indices, d (M, 3)
    node-minus-point offsets, valid (M, 3).
    """
    c = np.floor(X + 0.5).astype(np.int64)
    raw = c[:, None] + np.arange(-1, 2)[None, :]
    d = raw - X[:, None]
    if periodic:
        return np.mod(raw, n), d, np.ones(raw.shape, dtype=bool)
    valid = (raw >= 0) & (raw < n)
    return np.clip(raw, 0, n - 1), d, valid


# ---------------------------------------------------------------- MLS

GAUSS_ALPHA = 0.4     # Gaussian weight exp(-(s / alpha)^2), s = |r| / h, shifted to vanish at s = 1


@dataclass(frozen=True)
class Transfer:
    """Lattice <-> marker transfer: kind "roma" (the kernel) or "mls"."""
    kind: str = "roma"
    weight: str = "cubic"     # MLS weight: "roma", "cubic" or "gauss"
    h: float = 1.3            # support half-width of the cubic and Gaussian weights


ROMA = Transfer()


def support(tr: Transfer) -> float:
    return 1.5 if tr.weight == "roma" else float(tr.h)


def weight(r, tr: Transfer):
    """1-D MLS weight w(r) and its derivative dw/dr.

    cubic spline (s = |r|/h): 2/3 - 4 s^2 + 4 s^3 for s <= 1/2,
    4/3 (1 - s)^3 for 1/2 < s < 1; Gaussian: (e^{-(s/a)^2} - e^{-1/a^2}) /
    (1 - e^{-1/a^2}) for s < 1; both zero for s >= 1.  "roma": the kernel."""
    r = np.asarray(r, dtype=np.float64)
    if tr.weight == "roma":
        return phi(r), dphi(r)
    h = float(tr.h)
    s = np.abs(r) / h
    sg = np.sign(r) / h
    w = np.zeros_like(s)
    dw = np.zeros_like(s)
    if tr.weight == "cubic":
        m1 = s <= 0.5
        m2 = (s > 0.5) & (s < 1.0)
        w[m1] = 2.0 / 3.0 - 4.0 * s[m1] ** 2 + 4.0 * s[m1] ** 3
        dw[m1] = (-8.0 * s[m1] + 12.0 * s[m1] ** 2) * sg[m1]
        w[m2] = 4.0 / 3.0 * (1.0 - s[m2]) ** 3
        dw[m2] = -4.0 * (1.0 - s[m2]) ** 2 * sg[m2]
    elif tr.weight == "gauss":
        a = GAUSS_ALPHA
        e1 = np.exp(-1.0 / (a * a))
        m = s < 1.0
        g = np.exp(-(s[m] / a) ** 2)
        w[m] = (g - e1) / (1.0 - e1)
        dw[m] = -2.0 * s[m] / (a * a) * g / (1.0 - e1) * sg[m]
    else:
        raise ValueError(f"unknown MLS weight {tr.weight!r}")
    return w, dw


def mls_shape(XY: np.ndarray, nx: int, ny: int, periodic_y: bool, tr: Transfer):
    """MLS shape functions on the 3x3 stencil of each point and their
    derivatives with respect to the point position.

    Returns ix (M, 3), iy (M, 3) node indices and phi, dphi_dX, dphi_dY, each
    (M, 3, 3) indexed [point, a, b] for node (ix[:, a], iy[:, b]).

    The basis is centred on the point, p(x) = (1, x - X, y - Y), the centre
    held fixed while differentiating (the shape functions do not depend on
    where the basis is centred), so p(X) = e1, dp/dX = e2, dp/dY = e3 and
      gamma = A^{-1} e1,               phi_j = W_j gamma . p_j
      gamma_X = A^{-1} (e2 - A_X gamma)
      dphi_j/dX = W_j gamma_X . p_j + (dW_j/dX) gamma . p_j
    with A_X = sum_j (dW_j/dX) p_j p_j^T (the moving-least-squares derivative
    of Belytschko, Lu and Gu's element-free Galerkin method), likewise in Y.
    A point with fewer than two stencil rows inside the support (possible only
    next to a wall) uses the basis (1, x - X): p_j has no third component and
    the third row and column of A are those of the identity."""
    XY = np.asarray(XY, dtype=np.float64)
    M = XY.shape[0]
    ix, dx, _ = stencil(XY[:, 0], nx, True)
    iy, dy, vy = stencil(XY[:, 1], ny, periodic_y)
    wx, dwx = weight(dx, tr)
    wy, dwy = weight(dy, tr)
    wy = wy * vy
    dwy = dwy * vy
    h = support(tr)
    rows_in = np.sum(vy & (np.abs(dy) / h < 1.0), axis=1)
    ky = (rows_in >= 2).astype(np.float64)                 # 0: drop the y term
    # nodes j = (a, b): weights, their X and Y derivatives, basis vectors
    W = wx[:, :, None] * wy[:, None, :]
    WX = -dwx[:, :, None] * wy[:, None, :]                  # d/dX w(x_a - X) = -w'
    WY = -wx[:, :, None] * dwy[:, None, :]
    P = np.zeros((M, 3, 3, 3))
    P[..., 0] = 1.0
    P[..., 1] = dx[:, :, None]
    P[..., 2] = ky[:, None, None] * dy[:, None, :]
    A = np.einsum("mab,mabi,mabk->mik", W, P, P)
    AX = np.einsum("mab,mabi,mabk->mik", WX, P, P)
    AY = np.einsum("mab,mabi,mabk->mik", WY, P, P)
    A[:, 2, 2] += 1.0 - ky
    e = np.eye(3)
    gam = np.linalg.solve(A, np.broadcast_to(e[0], (M, 3))[..., None])[..., 0]
    rhsX = e[1][None, :] - np.einsum("mik,mk->mi", AX, gam)
    rhsY = ky[:, None] * e[2][None, :] - np.einsum("mik,mk->mi", AY, gam)
    gX = np.linalg.solve(A, rhsX[..., None])[..., 0]
    gY = np.linalg.solve(A, rhsY[..., None])[..., 0]
    gp = np.einsum("mi,mabi->mab", gam, P)
    ph = W * gp
    dphX = W * np.einsum("mi,mabi->mab", gX, P) + WX * gp
    dphY = W * np.einsum("mi,mabi->mab", gY, P) + WY * gp
    return ix, iy, ph, dphX, dphY


def _weights(XY: np.ndarray, nx: int, ny: int, periodic_y: bool):
    ix, dx, vx = stencil(XY[:, 0], nx, True)
    iy, dy, vy = stencil(XY[:, 1], ny, periodic_y)
    return ix, iy, dx, dy, vx, vy


def interpolate(field: np.ndarray, XY: np.ndarray, periodic_y: bool = False,
                tr: Transfer = ROMA) -> np.ndarray:
    """U_k = sum over the 3x3 stencil of field(x_j) delta(x_j - X_k) (or of
    field(x_j) phi_j(X_k) with the MLS transfer).  field: (ny, nx)."""
    ny, nx = field.shape
    if tr.kind == "mls":
        ix, iy, ph, _, _ = mls_shape(XY, nx, ny, periodic_y, tr)
        out = np.zeros(XY.shape[0])
        for a in range(3):
            for b in range(3):
                out += field[iy[:, b], ix[:, a]] * ph[:, a, b]
        return out
    ix, iy, dx, dy, vx, vy = _weights(XY, nx, ny, periodic_y)
    wx = phi(dx)
    wy = phi(dy) * vy
    out = np.zeros(XY.shape[0])
    for a in range(3):
        for b in range(3):
            out += field[iy[:, b], ix[:, a]] * wx[:, a] * wy[:, b]
    return out


def interpolate_gradient(field: np.ndarray, XY: np.ndarray, periodic_y: bool = False,
                         tr: Transfer = ROMA):
    """Gradient of the kernel interpolant with respect to the point position:
    d/dX_beta sum_j field_j delta(x_j - X) = -sum_j field_j phi'(.) phi(.)
    (with the MLS transfer: sum_j field_j dphi_j/dX_beta)."""
    ny, nx = field.shape
    if tr.kind == "mls":
        ix, iy, _, dX, dY = mls_shape(XY, nx, ny, periodic_y, tr)
        ddx = np.zeros(XY.shape[0])
        ddy = np.zeros(XY.shape[0])
        for a in range(3):
            for b in range(3):
                v = field[iy[:, b], ix[:, a]]
                ddx += v * dX[:, a, b]
                ddy += v * dY[:, a, b]
        return ddx, ddy
    ix, iy, dx, dy, vx, vy = _weights(XY, nx, ny, periodic_y)
    wx, wy = phi(dx), phi(dy) * vy
    gx_, gy_ = dphi(dx), dphi(dy) * vy
    ddx = np.zeros(XY.shape[0])
    ddy = np.zeros(XY.shape[0])
    for a in range(3):
        for b in range(3):
            v = field[iy[:, b], ix[:, a]]
            ddx -= v * gx_[:, a] * wy[:, b]
            ddy -= v * wx[:, a] * gy_[:, b]
    return ddx, ddy


def spread(F: np.ndarray, XY: np.ndarray, nx: int, ny: int, periodic_y: bool = False,
           tr: Transfer = ROMA) -> np.ndarray:
    """Eulerian force density sum_k F_k delta(x - X_k) (or sum_k F_k phi_j(X_k)
    with the MLS transfer); F: (M, 2).  Returns (2, ny, nx)."""
    out = np.zeros((2, ny, nx))
    if XY.shape[0] == 0:
        return out
    if tr.kind == "mls":
        ix, iy, ph, _, _ = mls_shape(XY, nx, ny, periodic_y, tr)
        for a in range(3):
            for b in range(3):
                np.add.at(out[0], (iy[:, b], ix[:, a]), F[:, 0] * ph[:, a, b])
                np.add.at(out[1], (iy[:, b], ix[:, a]), F[:, 1] * ph[:, a, b])
        return out
    ix, iy, dx, dy, vx, vy = _weights(XY, nx, ny, periodic_y)
    wx = phi(dx)
    wy = phi(dy) * vy
    for a in range(3):
        for b in range(3):
            w = wx[:, a] * wy[:, b]
            np.add.at(out[0], (iy[:, b], ix[:, a]), F[:, 0] * w)
            np.add.at(out[1], (iy[:, b], ix[:, a]), F[:, 1] * w)
    return out
