"""Vertex-vertex repulsion between different bodies (oracle), Sec. 2.2
"Particle-Particle Interaction", Eq. (repFor).  Test infrastructure only.

A vertex 1 at distance d from a vertex 2 of another body feels a purely
repulsive force of magnitude c sqrt(dx / d^5) (c = 1e-4 / (8 sqrt 2) in the
paper, lattice units dx = 1), directed along the inward normal of vertex 1.

Readings (the paper leaves these open):
  * every pair of vertices of two different bodies interacts, red cells and
    particles alike (Sec. 2.3 lists Eq. repFor among the internal forces of
    both body kinds); vertices of one body never repel each other;
  * only pairs closer than a cutoff r_c interact (default 2 dx; the
    expression itself has no cutoff);
  * the inward normal of vertex v is minus its outward vertex normal, the
    normalised sum of the outward normals of its two elements (the normal
    of the bending force); all close vertices of other bodies add their
    magnitudes along that one direction;
  * distances use the minimum image along x (periodic) and along y on a
    periodic lattice;
  * the force is evaluated at X^n with the other internal forces: red cells
    add it to the force they spread, soft particles to their vertex forces,
    rigid particles to their total force and torque (lever arm X_v - X_c).
"""
from __future__ import annotations

import numpy as np

from . import membrane

COEFF = 1e-4 / (8.0 * np.sqrt(2.0))   # Eq. (repFor), lattice units
CUTOFF = 2.0


def vertex_normals(xy: np.ndarray) -> np.ndarray:
    """Outward unit normal at each vertex: normalised sum of the normals of
    the elements v-1 -> v and v -> v+1."""
    _, _, n = membrane.elements(xy)
    s = n + np.roll(n, 1, axis=0)
    return s / np.hypot(s[:, 0], s[:, 1])[:, None]


def _min_image(d: np.ndarray, period: int) -> np.ndarray:
    return d - period * np.round(d / period)


def magnitudes(bodies_xy, coeff: float, cutoff: float, nx: int, ny: int,
               periodic_y: bool):
    """Per body, the summed magnitude c sum_j d_j^(-5/2) over the vertices j
    of all other bodies closer than `cutoff` (brute force over all pairs)."""
    out = []
    for a, A in enumerate(bodies_xy):
        s = np.zeros(A.shape[0])
        for b, B in enumerate(bodies_xy):
            if a == b:
                continue
            dx = _min_image(B[None, :, 0] - A[:, None, 0], nx)
            dy = B[None, :, 1] - A[:, None, 1]
            if periodic_y:
                dy = _min_image(dy, ny)
            d = np.hypot(dx, dy)
            close = d < cutoff
            s += np.where(close, coeff * np.sqrt(1.0 / np.where(close, d, 1.0) ** 5), 0.0).sum(axis=1)
        out.append(s)
    return out


def forces(bodies_xy, coeff: float, cutoff: float, nx: int, ny: int, periodic_y: bool):
    """Per body, the (nv, 2) repulsion forces: magnitude times inward normal."""
    mags = magnitudes(bodies_xy, coeff, cutoff, nx, ny, periodic_y)
    return [-(m[:, None] * vertex_normals(X)) for m, X in zip(mags, bodies_xy)]
