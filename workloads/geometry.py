"""Seeded synthetic geometry for the capillary workloads.

This module only *generates input data* (membrane vertex chains and their
placement); it contains none of the time-step arithmetic.  Both the FP64
oracle and the HIP library receive its output as plain vertex arrays and
each derives rest lengths, rest angles and rest areas on its own.

Shapes follow the set-up section of the paper:
  * red blood cell resting contour, Eq. (rbcShape): x = a*alpha*sin(q),
    y = a*(alpha/2)*(0.207 + 2.003 sin^2 q - 1.123 sin^4 q) cos(q),
    q in [-pi/2, 3pi/2], a = 1, alpha = cell radius;
  * particles: circles of radius r (0.5 um in the paper).
Vertices are returned counter-clockwise (the parametrisation above runs
clockwise), spaced at equal arc length.
"""
from __future__ import annotations

import numpy as np


def _resample_equal_arc(px: np.ndarray, py: np.ndarray, n: int) -> np.ndarray:
    """Resample a closed, densely sampled curve at n points of equal arc length."""
    seg = np.hypot(np.diff(np.append(px, px[0])), np.diff(np.append(py, py[0])))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    total = s[-1]
    t = np.arange(n) * (total / n)
    cx = np.append(px, px[0])
    cy = np.append(py, py[0])
    return np.stack([np.interp(t, s, cx), np.interp(t, s, cy)], axis=1)


def rbc_contour(alpha: float, n: int, dense: int = 40000) -> np.ndarray:
    """RBC resting contour (Eq. rbcShape) centred at the origin, long axis on x.

    Returns an (n, 2) float64 array, counter-clockwise, equal arc spacing.
    """
    q = np.linspace(-0.5 * np.pi, 1.5 * np.pi, dense, endpoint=False)
    s = np.sin(q)
    x = alpha * s
    y = 0.5 * alpha * (0.207 + 2.003 * s**2 - 1.123 * s**4) * np.cos(q)
    # the parametrisation is clockwise: reverse it
    x = x[::-1].copy()
    y = y[::-1].copy()
    pts = _resample_equal_arc(x, y, n)
    # start the chain at the left tip for reproducibility
    k = int(np.argmin(pts[:, 0]))
    return np.roll(pts, -k, axis=0)


def circle(r: float, n: int) -> np.ndarray:
    """Regular counter-clockwise n-gon of circumradius r centred at the origin."""
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def place(shape: np.ndarray, angle: float, centre) -> np.ndarray:
    """Rigidly rotate (counter-clockwise by angle) and translate a vertex chain."""
    c, s = np.cos(angle), np.sin(angle)
    R = np.array([[c, -s], [s, c]])
    return shape @ R.T + np.asarray(centre, dtype=np.float64)[None, :]


def signed_area(xy: np.ndarray) -> float:
    """Signed polygon area (positive for counter-clockwise); used to validate inputs."""
    x, y = xy[:, 0], xy[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def _inside(xy: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Even-odd point-in-polygon test for arrays of points."""
    x0, y0 = xy[:, 0], xy[:, 1]
    x1, y1 = np.roll(x0, -1), np.roll(y0, -1)
    inside = np.zeros(px.shape, dtype=bool)
    for a, b, c, d in zip(x0, y0, x1, y1):
        cond = (b > py) != (d > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xi = a + (py - b) * (c - a) / (d - b)
        inside ^= cond & (px < xi)
    return inside


def _inside_rows(xy: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Even-odd test on the raster xs (columns) x ys (rows); the same
    crossing abscissae and comparisons as `_inside`, organised per row."""
    x0, y0 = xy[:, 0], xy[:, 1]
    x1, y1 = np.roll(x0, -1), np.roll(y0, -1)
    out = np.zeros((ys.size, xs.size), dtype=bool)
    for r, yv in enumerate(ys):
        cond = (y0 > yv) != (y1 > yv)
        if not cond.any():
            continue
        a, b, c, d = x0[cond], y0[cond], x1[cond], y1[cond]
        xi = np.sort(a + (yv - b) * (c - a) / (d - b))
        # number of crossings with xs < xi
        n_right = xi.size - np.searchsorted(xi, xs, side="right")
        out[r] = (n_right & 1).astype(bool)
    return out


class Occupancy:
    """Raster occupancy of a periodic-x channel used for non-overlapping placement.

    A body is accepted if its region dilated by `gap` lattice units touches
    neither an already placed body nor the walls (y < gap or y > ny-1-gap).
    """

    def __init__(self, nx: int, ny: int, res: float = 1.0):
        self.nx, self.ny, self.res = nx, ny, res
        self.gx = int(np.ceil(nx / res))
        self.gy = int(np.ceil(ny / res))
        self.mask = np.zeros((self.gy, self.gx), dtype=bool)

    def _cells(self, xy: np.ndarray, gap: float):
        lo = xy.min(axis=0) - gap
        hi = xy.max(axis=0) + gap
        ix = np.arange(int(np.floor(lo[0] / self.res)), int(np.ceil(hi[0] / self.res)) + 1)
        iy = np.arange(int(np.floor(lo[1] / self.res)), int(np.ceil(hi[1] / self.res)) + 1)
        xs, ys = ix * self.res, iy * self.res
        PX, PY = np.meshgrid(xs, ys)
        ins = _inside_rows(xy, xs, ys)
        # dilation: any cell within `gap` of a vertex; only the window of
        # cells around each vertex can qualify
        near = np.zeros_like(ins)
        k = int(np.ceil(2.0 * gap / self.res)) + 3
        bx = np.floor((xy[:, 0] - gap) / self.res).astype(np.int64) - 1 - ix[0]
        by = np.floor((xy[:, 1] - gap) / self.res).astype(np.int64) - 1 - iy[0]
        off = np.arange(k)
        cx = np.clip(bx[:, None] + off[None, :], 0, ix.size - 1)        # (nv, k)
        cy = np.clip(by[:, None] + off[None, :], 0, iy.size - 1)
        dx2 = (xs[cx] - xy[:, 0:1]) ** 2                                  # (nv, k)
        dy2 = (ys[cy] - xy[:, 1:2]) ** 2
        hit = (dy2[:, :, None] + dx2[:, None, :]) <= gap * gap           # (nv, k, k)
        v, jy, jx = np.nonzero(hit)
        near[cy[v, jy], cx[v, jx]] = True
        sel = (ins | near).ravel()
        return ix, iy, PX.ravel()[sel], PY.ravel()[sel], sel.reshape(PX.shape)

    def try_add(self, xy: np.ndarray, gap: float) -> bool:
        ix, iy, px, py, sel = self._cells(xy, gap)
        if py.min() < 0.0 or py.max() > self.ny - 1:
            return False
        cx = np.mod(np.round(px / self.res).astype(np.int64), self.gx)
        cy = np.round(py / self.res).astype(np.int64)
        if self.mask[cy, cx].any():
            return False
        self.mask[cy, cx] = True
        return True
