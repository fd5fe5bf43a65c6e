"""One time step of the hybrid kinematic/dynamic LB-IB method (oracle).

State: post-collision populations f* (9, ny, nx); per body the vertex
positions at this and the previous time level; rigid-body centre, angle
and velocity history; the ligand-to-receptor bond table; the step counter.

Order of the sub-steps within step n (the paper does not fix it; this is
the reading used everywhere in this project):
  1. bonds: rupture then formation at the positions X^n;
  2. membrane forces at X^n (Eqs. strainFor, bendFor, areaFor), adhesion
     springs (Eq. adhFor) and, when enabled, the repulsion between vertices
     of different bodies (Eq. repFor, see repulsion.py);
  3. particles: probe loads from the pre-forcing fluid state, new
     positions X^{n+1} and velocities, weak-coupling forces (Sec. 2.3;
     soft vertices impose their displacement velocity, see particles.py);
  4. spreading: Eulerian force = uniform drive g + RBC forces at X^n +
     particle coupling forces at X^n;
  5. lattice Boltzmann collide-and-stream with that force (Sec. 2.1, 2.2);
     the half-force velocity u^n of this step is the physical field;
  6. red cells: kinematic IB, X^{n+1} = 2/3 (2 X^n - X^{n-1}/2 + U dt) with
     U = u^n interpolated at X^n (Eq. kinematicPos; forward Euler on the
     first step).  Particles adopt the positions from 3.
"""
from __future__ import annotations

import numpy as np

from . import adhesion, ib, lattice, membrane, particles, repulsion

RBC_KINEMATIC = 0
PARTICLE_SOFT = 1
PARTICLE_RIGID = 2


class BodyState:
    def __init__(self, kind, xy, ks, kb, ka, p_ref, density_ratio, sigma, ligand_stride):
        self.kind = int(kind)
        self.X = np.array(xy, dtype=np.float64)
        self.Xm = self.X.copy()
        self.nv = self.X.shape[0]
        # stress-free state = the given shape
        self.l0, _, _ = membrane.elements(self.X)
        self.theta0 = membrane.turning_angles(self.X)
        self.A0 = membrane.area(self.X)
        self.ks, self.kb, self.ka, self.p_ref = float(ks), float(kb), float(ka), float(p_ref)
        self.sigma = float(sigma)
        self.mass = float(density_ratio) * particles.RHO0 * self.A0
        self.mv = self.mass / self.nv
        self.ligands = (np.arange(0, self.nv, ligand_stride) if ligand_stride > 0
                        else np.zeros(0, dtype=np.int64))
        if self.kind == PARTICLE_RIGID:
            self.Xc = self.X.mean(axis=0)
            self.r0 = self.X - self.Xc[None, :]
            self.theta = 0.0
            self.inertia = 0.5 * self.mass * float(np.mean(np.sum(self.r0 ** 2, axis=1)))
            self.U = np.zeros(2)
            self.Um = np.zeros(2)
            self.Om = 0.0
            self.Omm = 0.0


class Sim:
    """FP64 reference time stepper; `step(k)` advances k time steps."""

    def __init__(self, wl):
        self.nx, self.ny = int(wl.nx), int(wl.ny)
        self.tau = float(wl.tau)
        self.nu = (self.tau - 0.5) / 3.0
        self.gx, self.gy = float(wl.gx), float(wl.gy)
        self.periodic_y = bool(wl.periodic_y)
        self.seed = int(wl.seed)
        self.instance = int(wl.instance)
        rho0 = np.ones((self.ny, self.nx)) if wl.rho0 is None else np.array(wl.rho0, dtype=np.float64)
        u0 = np.zeros((2, self.ny, self.nx)) if wl.u0 is None else np.array(wl.u0, dtype=np.float64)
        self.f = lattice.equilibrium(rho0, u0[0], u0[1])
        self.bodies = [BodyState(b.kind, b.xy, b.ks, b.kb, b.ka, b.p_ref, b.density_ratio,
                                 b.sigma, b.ligand_stride) for b in wl.bodies]
        self.lig_body = np.array([bi for bi, b in enumerate(self.bodies) for _ in b.ligands],
                                 dtype=np.int64)
        self.lig_elem = np.array([e for b in self.bodies for e in b.ligands], dtype=np.int64)
        self.l2r = -np.ones(len(self.lig_body), dtype=np.int64)
        self.receptors = [np.array(wl.receptors[0], dtype=np.float64),
                          np.array(wl.receptors[1], dtype=np.float64)]
        a = wl.adhesion
        self.bond_params = adhesion.BondParams(a.y_cr, a.y_eq, a.kf0_dt, a.kr0_dt,
                                               a.sigma_ts_frac, a.kbt)
        self.freeze_topology = bool(a.freeze_topology)
        # walls: halfway bounce-back at -1/2 and ny - 1/2, or the paper's
        # Zou-He velocity walls on the node rows 0 and ny - 1 (wet nodes)
        self.wet_walls = getattr(wl, "walls", "bounce-back") == "zou-he" and not self.periodic_y
        self.u_wall = tuple(float(u) for u in getattr(wl, "u_wall", (0.0, 0.0)))
        self.y_walls = (0.0, self.ny - 1.0) if self.wet_walls else None
        self.rep_coeff = float(getattr(wl, "repulsion", 0.0))
        self.rep_cutoff = float(getattr(wl, "repulsion_cutoff", repulsion.CUTOFF))
        # lattice <-> marker transfer: the Roma kernel or the general MLS fit
        self.tr = (ib.Transfer("mls", getattr(wl, "mls_weight", "cubic"),
                               float(getattr(wl, "mls_support", 1.3)))
                   if getattr(wl, "transfer", "roma") == "mls" else ib.ROMA)
        # velocity the weak coupling imposes at a soft-particle vertex:
        # "displacement" (X^{n+1} - X^n, the reading used everywhere) or
        # "verlet" (the second-order difference of Eq. verletVel, kept so
        # that a test can show why the first-order form is used)
        self.soft_velocity = "displacement"
        self.n = 0
        self.ties = 0
        self.rho = rho0.copy()
        self.ux, self.uy = u0[0].copy(), u0[1].copy()
        self.marker_force = [np.zeros((b.nv, 2)) for b in self.bodies]

    # ------------------------------------------------------------ helpers
    def ligand_centroids(self):
        c = np.zeros((len(self.lig_body), 2))
        for k, (bi, e) in enumerate(zip(self.lig_body, self.lig_elem)):
            X = self.bodies[bi].X
            c[k] = 0.5 * (X[e] + X[(e + 1) % X.shape[0]])
        return c

    def receptor(self, r):
        n0 = len(self.receptors[0])
        return (self.receptors[0][r], 0) if r < n0 else (self.receptors[1][r - n0], 1)

    def adhesion_element_forces(self, bi: int) -> np.ndarray:
        b = self.bodies[bi]
        out = np.zeros((b.nv, 2))
        if len(b.ligands) == 0:
            return out
        _, _, n = membrane.elements(b.X)
        c = membrane.centroids(b.X)
        for k in np.nonzero(self.lig_body == bi)[0]:
            r = int(self.l2r[k])
            if r < 0:
                continue
            e = int(self.lig_elem[k])
            xr, wall = self.receptor(r)
            out[e] += adhesion.spring_force(c[e], n[e], xr, wall, b.sigma,
                                            self.bond_params.y_eq, self.nx, self.ny, self.y_walls)
        return out

    # ------------------------------------------------------------ step
    def step(self, k: int = 1):
        for _ in range(int(k)):
            self._step_once()

    def _step_once(self):
        nx, ny, py = self.nx, self.ny, self.periodic_y
        first = self.n == 0
        # 1. bonds
        if len(self.l2r) and not self.freeze_topology:
            sig = np.array([self.bodies[bi].sigma for bi in self.lig_body])
            self.l2r, t = adhesion.bond_update(self.n, self.ligand_centroids(), sig, self.l2r,
                                               self.receptors, nx, ny, self.bond_params,
                                               self.seed, self.instance, self.y_walls)
            self.ties += t
        # pre-forcing fluid state of this step (streamed populations, drive
        # only; velocity walls set with the drive as the node force)
        fs = lattice.stream(self.f, py, self.wet_walls)
        fpre = (lattice.zou_he(fs, self.gx, self.gy, *self.u_wall) if self.wet_walls else fs)
        rho_s = lattice.density(fpre)
        jx, jy = lattice.momentum(fpre)
        ux_s = (jx + 0.5 * self.gx) / rho_s
        uy_s = (jy + 0.5 * self.gy) / rho_s
        # 2-3. forces and particle motion
        if self.rep_coeff > 0.0:
            frep = repulsion.forces([b.X for b in self.bodies], self.rep_coeff, self.rep_cutoff,
                                    nx, ny, py)
        else:
            frep = [np.zeros((b.nv, 2)) for b in self.bodies]
        Xnext = []
        for bi, b in enumerate(self.bodies):
            if b.kind == RBC_KINEMATIC:
                F = membrane.internal_force(b.X, b.l0, b.theta0, b.A0, b.ks, b.kb, b.ka, b.p_ref)
                F = F + frep[bi]
                self.marker_force[bi] = F
                Xnext.append(None)
                continue
            fel = particles.hydro_element_forces(b.X, rho_s, ux_s, uy_s, self.nu, py, self.tr)
            fel = fel + self.adhesion_element_forces(bi)
            U0 = np.stack([ib.interpolate(ux_s, b.X, py, self.tr),
                           ib.interpolate(uy_s, b.X, py, self.tr)], axis=1)
            ds = particles.marker_weights(b.X)
            if b.kind == PARTICLE_SOFT:
                Fv = (membrane.internal_force(b.X, b.l0, b.theta0, b.A0, b.ks, b.kb, b.ka, b.p_ref)
                      + membrane.share_to_vertices(fel) + frep[bi])
                Xn1 = b.X + U0 + 0.5 * Fv / b.mv
                if self.soft_velocity == "verlet" and not first:
                    Un1 = 1.5 * Xn1 - 2.0 * b.X + 0.5 * b.Xm      # Eq. verletVel
                else:
                    # velocity imposed by the weak coupling: displacement of the step
                    Un1 = Xn1 - b.X
            else:
                Ftot = fel.sum(axis=0) + frep[bi].sum(axis=0)
                c = membrane.centroids(b.X)
                Mtot = float(np.sum(particles.cross2(c - b.Xc[None, :], fel))
                             + np.sum(particles.cross2(b.X - b.Xc[None, :], frep[bi])))
                U = particles.bdf2(b.U, b.Um, Ftot / b.mass, first)
                Om = particles.bdf2(b.Om, b.Omm, Mtot / b.inertia, first)
                b.Um, b.U = b.U, U
                b.Omm, b.Om = b.Om, Om
                b.Xc = b.Xc + U
                b.theta = b.theta + Om
                Xn1 = b.Xc[None, :] + b.r0 @ particles.rotation(b.theta).T
                rel = Xn1 - b.Xc[None, :]
                Un1 = U[None, :] + Om * np.stack([-rel[:, 1], rel[:, 0]], axis=1)
            self.marker_force[bi] = particles.direct_forcing(Un1, U0, ds)
            Xnext.append(Xn1)
        # 4. spreading at X^n
        if self.bodies:
            XY = np.concatenate([b.X for b in self.bodies])
            F = np.concatenate(self.marker_force)
            FE = ib.spread(F, XY, nx, ny, py, self.tr)
        else:
            FE = np.zeros((2, ny, nx))
        FE[0] += self.gx
        FE[1] += self.gy
        # 5. lattice Boltzmann (velocity walls set with the full node force)
        if self.wet_walls:
            fpre = lattice.zou_he(fs, FE[0], FE[1], *self.u_wall)
        self.f, self.rho, self.ux, self.uy = lattice.collide(fpre, FE[0], FE[1], self.tau)
        # 6. marker advance
        for bi, b in enumerate(self.bodies):
            if b.kind == RBC_KINEMATIC:
                U = np.stack([ib.interpolate(self.ux, b.X, py, self.tr),
                              ib.interpolate(self.uy, b.X, py, self.tr)], axis=1)
                Xn1 = b.X + U if first else (2.0 / 3.0) * (2.0 * b.X - 0.5 * b.Xm + U)
            else:
                Xn1 = Xnext[bi]
            b.Xm = b.X
            b.X = Xn1
        self.n += 1

    # ------------------------------------------------------------ readback
    def fields(self):
        return self.rho, self.ux, self.uy

    def markers(self, bi: int) -> np.ndarray:
        return self.bodies[bi].X

    def all_markers(self) -> np.ndarray:
        return np.concatenate([b.X for b in self.bodies]) if self.bodies else np.zeros((0, 2))
