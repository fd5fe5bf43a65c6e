"""Ligand-receptor bonds between particles and walls (oracle).

Sec. 2.2 "Wall-Particle Interaction" and Sec. 3: ligands sit on the
particle boundary with density rho_L = 0.5, receptors are spread uniformly
on the walls; a bond is a linear spring F_l = sigma (y_l - y_eq) n_l
(Eq. adhFor), y_eq = y_cr / 2, evaluated at the element centroid and
shared equally by the element's two vertices; a bond can form only when
the boundary is closer to the wall than y_cr; formation and rupture are
stochastic with affinity k_f / k_r0 = 8.5e3.

The probability functions themselves are deferred by the paper to an
earlier work; the reading used is Bell/Dembo-type kinetics:
  k_f = k_f0 exp(-sigma_ts (y - y_eq)^2 / (2 kBT)),
  k_r = k_r0 exp((sigma - sigma_ts) (y - y_eq)^2 / (2 kBT)),
  P = 1 - exp(-k dt),
with sigma_ts = sigma_ts_frac * sigma.

Readings for what the text leaves open:
  * ligands on elements l with l % stride == 0 (stride 2 = every other);
  * element centroid c_l, outward element normal n_l; y_l = |c_l - r|,
    minimum image in x; wall distance d_l = min(c_y + 1/2, ny - 1/2 - c_y);
  * each step: rupture pass over bonded ligands in ascending global id,
    then formation pass over ligands free at the start of the step, in
    ascending id, restricted to d_l < y_cr; the candidate receptor is the
    nearest free one on the nearer wall (|dx| minimum image, ties to the
    lower receptor index); one bond per ligand and per receptor;
  * uniforms from Philox4x32-10 with counter (step, ligand id, purpose,
    instance): purpose 0 = formation, 1 = rupture.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import philox

TIE_BAND = 1e-12


@dataclass
class BondParams:
    y_cr: float
    y_eq: float
    kf0_dt: float
    kr0_dt: float
    sigma_ts_frac: float
    kbt: float


def wrap_x(cx: float, nx: int) -> float:
    return cx - nx * math.floor(cx / nx)


def min_image(xr: float, cx_wrapped: float, nx: int) -> float:
    d = xr - cx_wrapped
    if d > 0.5 * nx:
        d -= nx
    elif d < -0.5 * nx:
        d += nx
    return d


def wall_y(wall: int, ny: int, y_walls=None) -> float:
    """Wall positions: -1/2 and ny - 1/2 (halfway bounce-back), or the given
    pair (velocity walls on the node rows: 0 and ny - 1)."""
    if y_walls is not None:
        return float(y_walls[wall])
    return -0.5 if wall == 0 else ny - 0.5


def nearer_wall(cy: float, ny: int, y_walls=None):
    d0 = cy - wall_y(0, ny, y_walls)
    d1 = wall_y(1, ny, y_walls) - cy
    return (0, d0) if d0 <= d1 else (1, d1)


def bond_length(c, xr: float, wall: int, nx: int, ny: int, y_walls=None) -> float:
    dx = min_image(xr, wrap_x(c[0], nx), nx)
    dy = c[1] - wall_y(wall, ny, y_walls)
    return math.sqrt(dx * dx + dy * dy)


def formation_probability(y: float, sigma: float, p: BondParams) -> float:
    s_ts = p.sigma_ts_frac * sigma
    kf = p.kf0_dt * math.exp(-s_ts * (y - p.y_eq) ** 2 / (2.0 * p.kbt))
    return 1.0 - math.exp(-kf)


def rupture_probability(y: float, sigma: float, p: BondParams) -> float:
    s_ts = p.sigma_ts_frac * sigma
    kr = p.kr0_dt * math.exp((sigma - s_ts) * (y - p.y_eq) ** 2 / (2.0 * p.kbt))
    return 1.0 - math.exp(-kr)


def bond_update(step: int, lig_c, lig_sigma, lig_to_rec, receptors, nx: int, ny: int,
                p: BondParams, seed: int, instance: int = 0, y_walls=None):
    """One rupture-then-formation pass.

    lig_c: (N_L, 2) ligand centroids at this time level; lig_sigma: (N_L,)
    spring constant of each ligand's body; lig_to_rec: (N_L,) int, -1 free,
    else global receptor index (wall 0 receptors first, then wall 1);
    receptors: [x_wall0 (n0,), x_wall1 (n1,)].
    Returns the new lig_to_rec and the number of draws within TIE_BAND.
    """
    n0 = len(receptors[0])
    nrec = n0 + len(receptors[1])
    l2r = np.array(lig_to_rec, dtype=np.int64).copy()
    rec_taken = np.zeros(nrec, dtype=bool)
    rec_taken[l2r[l2r >= 0]] = True
    free_at_start = l2r < 0
    ties = 0

    def rec_pos(r):
        return (receptors[0][r], 0) if r < n0 else (receptors[1][r - n0], 1)

    # rupture
    for l in range(len(l2r)):
        r = int(l2r[l])
        if r < 0:
            continue
        xr, wall = rec_pos(r)
        y = bond_length(lig_c[l], xr, wall, nx, ny, y_walls)
        P = rupture_probability(y, lig_sigma[l], p)
        u = philox.uniform(seed, step, l, philox.PURPOSE_RUPTURE, instance)
        ties += abs(u - P) < TIE_BAND
        if u < P:
            l2r[l] = -1
            rec_taken[r] = False
    # formation
    for l in range(len(l2r)):
        if not free_at_start[l]:
            continue
        wall, d = nearer_wall(lig_c[l][1], ny, y_walls)
        if not d < p.y_cr:
            continue
        xs = receptors[wall]
        off = 0 if wall == 0 else n0
        cxw = wrap_x(lig_c[l][0], nx)
        best, bestd = -1, math.inf
        for k in range(len(xs)):
            if rec_taken[off + k]:
                continue
            dd = abs(min_image(xs[k], cxw, nx))
            if dd < bestd:
                best, bestd = k, dd
        if best < 0:
            continue
        y = bond_length(lig_c[l], xs[best], wall, nx, ny, y_walls)
        P = formation_probability(y, lig_sigma[l], p)
        u = philox.uniform(seed, step, l, philox.PURPOSE_FORM, instance)
        ties += abs(u - P) < TIE_BAND
        if u < P:
            l2r[l] = off + best
            rec_taken[off + best] = True
    return l2r, ties


def spring_force(c, n, xr: float, wall: int, sigma: float, y_eq: float, nx: int, ny: int,
                 y_walls=None):
    """Eq. (adhFor): F = sigma (y_l - y_eq) n_l at the element centroid."""
    y = bond_length(c, xr, wall, nx, ny, y_walls)
    return sigma * (y - y_eq) * np.asarray(n, dtype=np.float64)
