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
"""
from __future__ import annotations

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


def _weights(XY: np.ndarray, nx: int, ny: int, periodic_y: bool):
    ix, dx, vx = stencil(XY[:, 0], nx, True)
    iy, dy, vy = stencil(XY[:, 1], ny, periodic_y)
    return ix, iy, dx, dy, vx, vy


def interpolate(field: np.ndarray, XY: np.ndarray, periodic_y: bool = False) -> np.ndarray:
    """U_k = sum over the 3x3 stencil of field(x_j) delta(x_j - X_k).  field: (ny, nx)."""
    ny, nx = field.shape
    ix, iy, dx, dy, vx, vy = _weights(XY, nx, ny, periodic_y)
    wx = phi(dx)
    wy = phi(dy) * vy
    out = np.zeros(XY.shape[0])
    for a in range(3):
        for b in range(3):
            out += field[iy[:, b], ix[:, a]] * wx[:, a] * wy[:, b]
    return out


def interpolate_gradient(field: np.ndarray, XY: np.ndarray, periodic_y: bool = False):
    """Gradient of the kernel interpolant with respect to the point position:
    d/dX_beta sum_j field_j delta(x_j - X) = -sum_j field_j phi'(.) phi(.)."""
    ny, nx = field.shape
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


def spread(F: np.ndarray, XY: np.ndarray, nx: int, ny: int, periodic_y: bool = False) -> np.ndarray:
    """Eulerian force density sum_k F_k delta(x - X_k); F: (M, 2).  Returns (2, ny, nx)."""
    out = np.zeros((2, ny, nx))
    if XY.shape[0] == 0:
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
