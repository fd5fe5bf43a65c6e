"""Dynamic immersed-boundary motion of rigid and soft particles (oracle).

Sec. 2.2 "Hydrodynamics Stresses": per element, pressure load
F^p = -p_l n_l l_l (Eq. hydroForP) and viscous load F^tau = (tau_l . n_l) l_l
(Eq. hydroForNu), with p and the velocity derivatives taken at a probe
1.2 dx along the outward normal from the element centroid and attributed
to the centroid; element loads are shared equally by the two vertices.
Sec. 2.3: soft particles integrate Newton's law per vertex (Eq. newtonSoft)
with the Verlet position update seeded by the interpolated fluid velocity
(Eq. verletPos); rigid particles sum
loads into a force and a moment and advance U and Omega with BDF2
(Eqs. linearVelRig, angularVelRig).  No-slip is imposed weakly.

Readings for what the text leaves open:
  * probe quantities come from the pre-forcing fluid state of this step:
    rho* = sum f_i and u* = (sum f_i e_i + g/2)/rho* of the streamed
    populations, g the uniform driving force; p = cs^2 (rho* - rho0);
    velocity gradient = gradient of the kernel (or MLS) interpolant;
    tau = rho0 nu (grad u + grad u^T);
  * with walls the probe ordinate is clamped to [1/2, ny - 3/2] so the
    probe stencil stays inside the fluid;
  * particle mass m = (rho_P/rho) rho0 A_0, spread uniformly over the
    vertices of a soft particle; rigid inertia I = m <|r_k|^2> / 2 about the
    vertex mean (a disc: m r^2 / 2); rigid positions advance as
    X_c += U dt, theta += Omega dt; first step uses forward Euler;
  * weak coupling: the marker velocity U_k^{n+1} of the particle is
    imposed through the Eulerian force F_k = 2 rho0 (U_k^{n+1} - u*(X_k^n)),
    spread at X_k^n with weight ds_k = (l_{k-1} + l_k)/2; the internal
    forces of a particle reach the fluid only through this term;
  * the imposed velocity of a soft-particle vertex is its displacement over
    the step, (X^{n+1} - X^n)/dt.  The second-order velocity of Eq.
    (verletVel), 3/2 X^{n+1} - 2 X^n + 1/2 X^{n-1}, reduces the coupling
    force to a difference of successive interpolated fluid velocities, a
    feedback with a unit eigenvalue that grows (about x1.2 per step) once a
    vertex sits in the half cell next to a wall; the displacement velocity
    is the first-order form of the same quantity and is stable there.
"""
from __future__ import annotations

import numpy as np

from . import ib, membrane
from .lattice import CS2

PROBE_LENGTH = 1.2
RHO0 = 1.0


def probe_points(xy: np.ndarray, ny: int, periodic_y: bool) -> np.ndarray:
    _, _, n = membrane.elements(xy)
    q = membrane.centroids(xy) + PROBE_LENGTH * n
    if not periodic_y:
        q[:, 1] = np.clip(q[:, 1], 0.5, ny - 1.5)
    return q


def hydro_element_forces(xy, rho_s, ux_s, uy_s, nu: float, periodic_y: bool,
                         tr: ib.Transfer = ib.ROMA) -> np.ndarray:
    """F^p + F^tau per element, (nv, 2)."""
    ny = rho_s.shape[0]
    length, _, n = membrane.elements(xy)
    q = probe_points(xy, ny, periodic_y)
    p = CS2 * (ib.interpolate(rho_s, q, periodic_y, tr) - RHO0)
    dudx, dudy = ib.interpolate_gradient(ux_s, q, periodic_y, tr)
    dvdx, dvdy = ib.interpolate_gradient(uy_s, q, periodic_y, tr)
    txx = 2.0 * RHO0 * nu * dudx
    tyy = 2.0 * RHO0 * nu * dvdy
    txy = RHO0 * nu * (dudy + dvdx)
    fx = (-p * n[:, 0] + txx * n[:, 0] + txy * n[:, 1]) * length
    fy = (-p * n[:, 1] + txy * n[:, 0] + tyy * n[:, 1]) * length
    return np.stack([fx, fy], axis=1)


def marker_weights(xy: np.ndarray) -> np.ndarray:
    """ds_k = (l_{k-1} + l_k) / 2."""
    length, _, _ = membrane.elements(xy)
    return 0.5 * (np.roll(length, 1) + length)


def direct_forcing(U_next: np.ndarray, U_star: np.ndarray, ds: np.ndarray) -> np.ndarray:
    """Spread force of the weak no-slip coupling, already multiplied by ds."""
    return (2.0 * RHO0 * (U_next - U_star)) * ds[:, None]


def bdf2(v, v_prev, rate, first: bool):
    """Eqs. (linearVelRig)/(angularVelRig): v^{n+1} = 2/3 (2 v^n - v^{n-1}/2 + rate dt)."""
    if first:
        return v + rate
    return (2.0 / 3.0) * (2.0 * v - 0.5 * v_prev + rate)


def rotation(theta: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s], [s, c]])


def cross2(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
