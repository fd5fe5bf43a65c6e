"""Per-body observables of a run (oracle), the quantities the paper reports in
Sec. 3 (margination and adhesion results).  Test infrastructure only.

An observation at step n records, for every body:
  * the centre of mass X_c = mean of the vertex positions (vertices carry
    equal masses: m_v = m / n_v);
  * the flow region of its lateral position eta = (y_c - y_lo) / (y_hi - y_lo)
    between the walls (y = -1/2 and n_y - 1/2 with halfway bounce-back, the
    node rows 0 and n_y - 1 with velocity walls): the cell-free layer eta <= 0.2 or
    eta >= 0.8, the intermediate zone 0.2 < eta < 0.3 or 0.7 < eta < 0.8,
    the bulk 0.3 <= eta <= 0.7 (Sec. 3, three flow regions);
  * r_max, the largest lateral displacement |y_c - y_c,0| from the release
    position seen so far (Sec. 3, <r_max>/H);
  * the centre-of-mass velocity over the interval since the previous
    observation, (X_c - X_c,prev) / (n - n_prev), and running sums of it (the
    rolling velocity u_roll and the lateral velocity, Sec. 3);
  * n_L, the number of its ligands holding a bond, and n_L0, that number at
    the first observation (Sec. 3, n_L / n_L0).

Readings (the paper defines the regions by open intervals that leave 0.2 and
0.8 unassigned, and gives the rest in words): the two boundaries belong to the
cell-free layer; the release position and n_L0 are those of the first
observation; velocities are per time step in lattice units (divide by u_max
for the paper's ratios).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

CFL, INTERMEDIATE, BULK = 0, 1, 2


def centre_of_mass(xy: np.ndarray) -> np.ndarray:
    return np.asarray(xy, dtype=np.float64).mean(axis=0)


def region(yc: float, ny: int, y_walls=None) -> int:
    """Flow region of a lateral position; walls at -1/2 and ny - 1/2, or at
    the given positions (velocity walls on the node rows 0 and ny - 1)."""
    lo, hi = (-0.5, ny - 0.5) if y_walls is None else y_walls
    eta = (yc - lo) / (hi - lo)
    if eta <= 0.2 or eta >= 0.8:
        return CFL
    if 0.3 <= eta <= 0.7:
        return BULK
    return INTERMEDIATE


@dataclass
class BodyObs:
    xc: float = 0.0
    yc: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    r_max: float = 0.0
    u_x: float = 0.0
    u_y: float = 0.0
    u_x_sum: float = 0.0
    u_y_sum: float = 0.0
    region: int = 0
    n_bonds: int = 0
    n_bonds0: int = 0
    n_obs: int = 0
    step_obs: int = 0


class Observer:
    """Accumulates observations of a sequence of states."""

    def __init__(self, n_bodies: int):
        self.obs = [BodyObs() for _ in range(n_bodies)]

    def observe(self, step: int, bodies_xy, bonds_per_body, ny: int, y_walls=None):
        for o, xy, nb in zip(self.obs, bodies_xy, bonds_per_body):
            c = centre_of_mass(xy)
            if o.n_obs == 0:
                o.x0, o.y0 = float(c[0]), float(c[1])
                o.n_bonds0 = int(nb)
            else:
                dn = step - o.step_obs
                if dn > 0:
                    o.u_x = (float(c[0]) - o.xc) / dn
                    o.u_y = (float(c[1]) - o.yc) / dn
                    o.u_x_sum += o.u_x
                    o.u_y_sum += o.u_y
            o.xc, o.yc = float(c[0]), float(c[1])
            o.r_max = max(o.r_max, abs(o.yc - o.y0))
            o.region = region(o.yc, ny, y_walls)
            o.n_bonds = int(nb)
            o.n_obs += 1
            o.step_obs = int(step)

    def observe_sim(self, sim):
        """Observation of an oracle `Sim` at its current step."""
        nb = np.zeros(len(sim.bodies), dtype=np.int64)
        for k, bi in enumerate(sim.lig_body):
            if sim.l2r[k] >= 0:
                nb[bi] += 1
        self.observe(sim.n, [b.X for b in sim.bodies], nb, sim.ny, sim.y_walls)
