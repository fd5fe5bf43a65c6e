"""Mass-spring membrane forces (oracle), Sec. 2.2 "Elastic Membrane Deformation".

A body is a closed chain of nv vertices x_0..x_{nv-1} listed counter-
clockwise; element l joins vertex l to vertex l+1 (mod nv).  Per element:
length l_l, unit tangent t_l = (x_{l+1} - x_l)/l_l and outward unit normal
n_l = (t_l,y, -t_l,x).  Forces are returned per vertex, shape (nv, 2).

  strain   (Eq. strainFor): F_1 = -k_s (l - l_0) r_12 / l on both ends,
           the gradient of V = k_s (l - l_0)^2 / 2 (Eq. strainPot);
  bending  (Eq. bendFor): with Delta = theta - theta_0 at vertex v,
           F_left = k_b Delta l_left/(l_left + l_right) n_v,
           F_v = -k_b Delta n_v, F_right = k_b Delta l_right/(l_left + l_right) n_v,
           where the sentence after the equation names l_right and l_left
           the lengths of the left and right edges, respectively: the
           neighbour across the shorter edge takes the larger share (the
           lever rule), and the three forces exert neither a net force nor
           a net moment;
  area     (Eq. areaFor): F_l = -k_a (1 - A/A_0) p_ref (n_l)^- l_l with
           (n_l)^- = -n_l, shared equally by the two vertices of l.

Readings: theta is the signed turning angle between consecutive unit
tangents, atan2(t_L x t_R, t_L . t_R); the vertex normal n_v is the
normalised sum of the two adjacent element normals; the enclosed area is
the exact polygon (shoelace) area, the Green's-theorem sum of the text.
"""
from __future__ import annotations

import numpy as np


def elements(xy: np.ndarray):
    """Element lengths (nv,), unit tangents (nv, 2) and outward normals (nv, 2)."""
    d = np.roll(xy, -1, axis=0) - xy
    length = np.hypot(d[:, 0], d[:, 1])
    t = d / length[:, None]
    n = np.stack([t[:, 1], -t[:, 0]], axis=1)
    return length, t, n


def centroids(xy: np.ndarray) -> np.ndarray:
    """Element centroids c_l = (x_l + x_{l+1}) / 2."""
    return 0.5 * (xy + np.roll(xy, -1, axis=0))


def turning_angles(xy: np.ndarray) -> np.ndarray:
    """theta_v between left element (v-1 -> v) and right element (v -> v+1)."""
    _, t, _ = elements(xy)
    tl = np.roll(t, 1, axis=0)
    tr = t
    cross = tl[:, 0] * tr[:, 1] - tl[:, 1] * tr[:, 0]
    dot = tl[:, 0] * tr[:, 0] + tl[:, 1] * tr[:, 1]
    return np.arctan2(cross, dot)


def area(xy: np.ndarray) -> float:
    """Enclosed (signed) area, positive for a counter-clockwise chain."""
    x, y = xy[:, 0], xy[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def strain_force(xy: np.ndarray, l0: np.ndarray, ks: float) -> np.ndarray:
    length, t, _ = elements(xy)
    fe = (ks * (length - l0))[:, None] * t       # force on the first vertex of each element
    F = fe.copy()                                # vertex l gets +fe_l
    F -= np.roll(fe, 1, axis=0)                  # vertex l+1 gets -fe_l
    return F


def strain_energy(xy: np.ndarray, l0: np.ndarray, ks: float) -> float:
    length, _, _ = elements(xy)
    return float(0.5 * ks * np.sum((length - l0) ** 2))


def bending_force(xy: np.ndarray, theta0: np.ndarray, kb: float) -> np.ndarray:
    length, _, n = elements(xy)
    nv = xy.shape[0]
    theta = turning_angles(xy)
    delta = theta - theta0
    len_left_edge = np.roll(length, 1)   # element v-1 -> v
    len_right_edge = length              # element v -> v+1
    # the symbols of Eq. bendFor: l_left is the right edge's length and
    # l_right the left edge's (the defining sentence's "respectively")
    l_left, l_right = len_right_edge, len_left_edge
    nsum = np.roll(n, 1, axis=0) + n
    nvert = nsum / np.hypot(nsum[:, 0], nsum[:, 1])[:, None]
    F = np.zeros((nv, 2))
    for v in range(nv):
        k = kb * delta[v]
        s = l_left[v] + l_right[v]
        F[(v - 1) % nv] += k * l_left[v] / s * nvert[v]
        F[v] -= k * nvert[v]
        F[(v + 1) % nv] += k * l_right[v] / s * nvert[v]
    return F


def area_element_force(xy: np.ndarray, A0: float, ka: float, p_ref: float) -> np.ndarray:
    """Per-element area penalty force F_l^a (before sharing to vertices)."""
    length, _, n = elements(xy)
    A = area(xy)
    return (ka * (1.0 - A / A0) * p_ref * length)[:, None] * n


def share_to_vertices(fel: np.ndarray) -> np.ndarray:
    """Element forces given half to each of the element's two vertices."""
    return 0.5 * fel + 0.5 * np.roll(fel, 1, axis=0)


def area_force(xy: np.ndarray, A0: float, ka: float, p_ref: float) -> np.ndarray:
    return share_to_vertices(area_element_force(xy, A0, ka, p_ref))


def internal_force(xy, l0, theta0, A0, ks, kb, ka, p_ref) -> np.ndarray:
    """Strain + bending + area forces on every vertex."""
    return (strain_force(xy, l0, ks) + bending_force(xy, theta0, kb)
            + area_force(xy, A0, ka, p_ref))
