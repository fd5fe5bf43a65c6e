"""D2Q9 BGK lattice Boltzmann with Guo forcing, FP64 (oracle).

Sec. 2.1 of the paper: discrete Boltzmann equation with single relaxation
time tau (Eq. BGK), viscosity nu = cs^2 (tau - 1/2) dt, cs^2 = 1/3,
moments rho = sum f_i, rho u = sum f_i e_i, second-order equilibrium
(Eq. feq), nine velocities and weights (Eq. GaussHermite).
Sec. 2.2: forced update (Eq. forcedBGK) with Guo's source term
(Eq. ForcingTerm) and half-force momentum rho u = sum f_i e_i + f/2.

Lattice units dt = dx = 1.  Arrays are indexed [i, y, x].

Readings where the text is garbled or silent:
  * Eq. (ForcingTerm) is read as (1 - 1/(2 tau)) w_i [(e_i - u)/cs^2 +
    (e_i . u) e_i / cs^4] . f, i.e. the prefactor multiplies the whole
    bracket (Guo et al.'s term);
  * the half-force momentum uses the total Eulerian force (body force plus
    immersed-boundary force);
  * walls: halfway bounce-back at y = -1/2 and y = ny - 1/2 (no-slip),
    x periodic.  An optional periodic-y mode removes the walls (tests).
    The paper's own wall condition, Zou-He velocity walls on the node rows
    y = 0 and y = ny - 1 (wet nodes, channel height ny - 1), is the other
    mode: see `zou_he`.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def velocities() -> np.ndarray:
    """Eq. (GaussHermite): e_0 = 0, e_1..4 on the axes, e_5..8 on the diagonals."""
    e = np.zeros((9, 2))
    for i in range(1, 5):
        a = (i - 1) * np.pi / 2.0
        e[i] = [np.cos(a), np.sin(a)]
    for i in range(5, 9):
        a = (2 * i - 9) * np.pi / 4.0
        e[i] = np.sqrt(2.0) * np.array([np.cos(a), np.sin(a)])
    return np.rint(e).astype(np.int64)


E = velocities()
W = np.array([4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4)
OPP = np.array([int(np.nonzero((E == -E[i]).all(axis=1))[0][0]) for i in range(9)])


def equilibrium(rho: np.ndarray, ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
    """Eq. (feq): w_i rho [1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u.u/(2 cs^2)]."""
    uu = ux * ux + uy * uy
    out = np.empty((9,) + rho.shape)
    for i in range(9):
        eu = E[i, 0] * ux + E[i, 1] * uy
        out[i] = W[i] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))
    return out


def guo_source(ux, uy, fx, fy, tau: float) -> np.ndarray:
    """Eq. (ForcingTerm): (1 - 1/(2 tau)) w_i [(e_i - u)/cs^2 + (e_i.u) e_i/cs^4] . f."""
    out = np.empty((9,) + np.shape(ux))
    pre = 1.0 - 1.0 / (2.0 * tau)
    for i in range(9):
        ex, ey = E[i]
        eu = ex * ux + ey * uy
        bx = (ex - ux) / CS2 + eu * ex / (CS2 * CS2)
        by = (ey - uy) / CS2 + eu * ey / (CS2 * CS2)
        out[i] = pre * W[i] * (bx * fx + by * fy)
    return out


def stream(fpost: np.ndarray, periodic_y: bool = False, wet_walls: bool = False) -> np.ndarray:
    """Pull streaming f_i(x) <- f*_i(x - e_i), x periodic.

    With walls, a population whose source node lies beyond the lattice is
    the opposite population reflected at the same node (halfway bounce-back,
    wall at rest), or with wet_walls unknown (NaN) until `zou_he` sets it.
    """
    ny = fpost.shape[1]
    fpre = np.empty_like(fpost)
    for i in range(9):
        ex, ey = E[i]
        fpre[i] = np.roll(np.roll(fpost[i], ex, axis=1), ey, axis=0)
        if not periodic_y:
            if ey == 1:      # source row y-1 does not exist for y = 0
                fpre[i, 0, :] = np.nan if wet_walls else fpost[OPP[i], 0, :]
            elif ey == -1:   # source row y+1 does not exist for y = ny-1
                fpre[i, ny - 1, :] = np.nan if wet_walls else fpost[OPP[i], ny - 1, :]
    return fpre


def zou_he(fpre: np.ndarray, fx, fy, u_lo: float, u_hi: float) -> np.ndarray:
    """Velocity walls on the node rows y = 0 and y = ny - 1 (Zou & He, the
    paper's wall condition, Sec. 2.1): the populations that would come from
    beyond the wall are set so that the node's half-force velocity is the
    wall velocity (u_w, 0), i.e. its bare momentum sum f e = rho u_w - F/2,
    with the density following from the known populations, and the
    non-equilibrium parts of the normal pair bounced back.

    Reading: with a force at the wall node, the prescribed velocity is the
    half-force velocity of Sec. 2.2 (the bare momentum carries -F/2).
    """
    f = fpre.copy()
    ny = f.shape[1]
    # bottom row: unknown 2 (+y), 5 (+x+y), 6 (-x+y)
    y = 0
    Fx, Fy = np.broadcast_to(fx, f.shape[1:])[y], np.broadcast_to(fy, f.shape[1:])[y]
    rho = f[0, y] + f[1, y] + f[3, y] + 2.0 * (f[4, y] + f[7, y] + f[8, y]) - 0.5 * Fy
    jx, jy = rho * u_lo - 0.5 * Fx, -0.5 * Fy
    d13 = f[1, y] - f[3, y]
    f[2, y] = f[4, y] + (2.0 / 3.0) * jy
    f[5, y] = f[7, y] - 0.5 * d13 + 0.5 * jx + jy / 6.0
    f[6, y] = f[8, y] + 0.5 * d13 - 0.5 * jx + jy / 6.0
    # top row: unknown 4 (-y), 7 (-x-y), 8 (+x-y)
    y = ny - 1
    Fx, Fy = np.broadcast_to(fx, f.shape[1:])[y], np.broadcast_to(fy, f.shape[1:])[y]
    rho = f[0, y] + f[1, y] + f[3, y] + 2.0 * (f[2, y] + f[5, y] + f[6, y]) + 0.5 * Fy
    jx, jy = rho * u_hi - 0.5 * Fx, -0.5 * Fy
    d13 = f[1, y] - f[3, y]
    f[4, y] = f[2, y] - (2.0 / 3.0) * jy
    f[7, y] = f[5, y] + 0.5 * d13 - 0.5 * jx - jy / 6.0
    f[8, y] = f[6, y] - 0.5 * d13 + 0.5 * jx - jy / 6.0
    return f


def density(f: np.ndarray) -> np.ndarray:
    return f.sum(axis=0)


def momentum(f: np.ndarray):
    jx = np.tensordot(E[:, 0].astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(E[:, 1].astype(np.float64), f, axes=(0, 0))
    return jx, jy


def velocity(f: np.ndarray, fx, fy):
    """rho and the half-force velocity u = (sum f e + f/2) / rho (Sec. 2.2)."""
    rho = density(f)
    jx, jy = momentum(f)
    return rho, (jx + 0.5 * fx) / rho, (jy + 0.5 * fy) / rho


def collide(fpre: np.ndarray, fx, fy, tau: float):
    """Eq. (forcedBGK) with dt = 1: f* = f - (f - f^eq)/tau + F_i."""
    rho, ux, uy = velocity(fpre, fx, fy)
    feq = equilibrium(rho, ux, uy)
    src = guo_source(ux, uy, fx, fy, tau)
    fpost = fpre - (fpre - feq) / tau + src
    return fpost, rho, ux, uy


def lb_step(fpost: np.ndarray, fx, fy, tau: float, periodic_y: bool = False):
    """One collide-and-stream: stream the stored post-collision populations,
    then relax with the Eulerian force field (fx, fy).

    Returns the new post-collision populations and the physical fields
    (rho, ux, uy) of this time level.
    """
    fpre = stream(fpost, periodic_y)
    return collide(fpre, fx, fy, tau)
