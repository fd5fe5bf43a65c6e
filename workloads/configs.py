"""Seeded synthetic workload descriptions for the capillary LB-IB step.

Each builder returns a plain `Workload` (lattice parameters, body vertex
chains, receptor positions, adhesion parameters) that both the FP64 oracle
and the HIP library consume as data.  Nothing here advances the method.

Lattice units throughout: dx = dt = 1, rho0 = 1, cs^2 = 1/3.

Parameter derivations (set-up section of the paper):
  * nu = (tau - 1/2)/3 (tau fixed at 1 in every computation of the paper);
  * centre-line velocity from Re = u_max H / nu = 1e-2, or from a Mach number;
  * membrane stiffness from the capillary number Ca = rho nu u_max / k_s;
  * bending constant from Eb = k_b / (k_s r^2) (0.05 for particles, 0 for RBCs);
  * bond spring constant sigma in units rho nu^2 / H; critical bond length
    25 nm, equilibrium length half of it;
  * affinity k_f / k_r0 = 8.5e3; particle to fluid density ratio 1.1.
The uniform body force that drives the plane Poiseuille flow is chosen so
that the centre-line velocity of the discrete steady state equals u_max
(for halfway bounce-back walls the discrete profile carries a slip term
(16 L - 3)/12, L = (tau - 1/2)^2, on top of the parabola).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import geometry

RBC_KINEMATIC = 0
PARTICLE_SOFT = 1
PARTICLE_RIGID = 2

SEED_BASE = 190700080  # seeds are SEED_BASE + config number (+ instance)

BOLTZMANN = 1.380649e-23

REPULSION_COEFF = 1e-4 / (8.0 * np.sqrt(2.0))  # Eq. repFor prefactor, lattice units


@dataclass
class Body:
    kind: int
    xy: np.ndarray            # (nv, 2) float64, counter-clockwise, stress-free shape
    ks: float = 0.0
    kb: float = 0.0
    ka: float = 1.0
    p_ref: float = 1.0 / 3.0
    density_ratio: float = 1.1
    sigma: float = 0.0         # bond spring constant, lattice units
    ligand_stride: int = 0     # 0: no ligands; 2: every other element


@dataclass
class Adhesion:
    y_cr: float = 0.5
    y_eq: float = 0.25
    kf0_dt: float = 1e-3
    kr0_dt: float = 1e-3 / 8.5e3
    sigma_ts_frac: float = 0.5
    kbt: float = 1.0
    freeze_topology: int = 0


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    tau: float = 1.0
    gx: float = 0.0
    gy: float = 0.0
    periodic_y: int = 0
    seed: int = SEED_BASE
    instance: int = 0
    bodies: List[Body] = field(default_factory=list)
    receptors: List[np.ndarray] = field(default_factory=lambda: [np.zeros(0), np.zeros(0)])
    adhesion: Adhesion = field(default_factory=Adhesion)
    walls: str = "bounce-back"          # or "zou-he": velocity walls on rows 0 and ny - 1
    u_wall: tuple = (0.0, 0.0)          # wall velocities along x (bottom, top), zou-he only
    repulsion: float = 0.0              # Eq. repFor coefficient (0: off; REPULSION_COEFF)
    repulsion_cutoff: float = 2.0       # pairs closer than this interact
    transfer: str = "roma"              # lattice <-> marker transfer: "roma" kernel or "mls"
    mls_weight: str = "cubic"           # MLS weight: "roma", "cubic" or "gauss"
    mls_support: float = 1.3            # MLS support half-width (square of side 2.6 dx)
    rho0: Optional[np.ndarray] = None   # (ny, nx) initial density, None -> 1
    u0: Optional[np.ndarray] = None     # (2, ny, nx) initial velocity, None -> 0
    steps: int = 1000
    dtype: str = "f32"

    @property
    def n_markers(self) -> int:
        return int(sum(b.xy.shape[0] for b in self.bodies))

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


# ---------------------------------------------------------------- units

def viscosity(tau: float) -> float:
    return (tau - 0.5) / 3.0


def poiseuille_force(u_max: float, ny: int, tau: float) -> float:
    """Body force whose discrete steady channel flow peaks at u_max."""
    nu = viscosity(tau)
    lam = (tau - 0.5) ** 2
    return 2.0 * nu * u_max / ((ny / 2.0) ** 2 + (16.0 * lam - 3.0) / 12.0)


def poiseuille_profile(g: float, ny: int, tau: float) -> np.ndarray:
    """Discrete steady profile u(y), y = 0..ny-1, walls at -1/2 and ny-1/2."""
    nu = viscosity(tau)
    lam = (tau - 0.5) ** 2
    y = np.arange(ny, dtype=np.float64)
    return g / (2.0 * nu) * ((y + 0.5) * (ny - 0.5 - y) + (16.0 * lam - 3.0) / 12.0)


def kbt_lattice(dx_m: float, nu_lu: float, nu_phys: float = 1.2e-6,
                rho_phys: float = 1000.0, temp: float = 310.0) -> float:
    """Thermal energy in lattice units for a 2D slab one lattice spacing deep."""
    dt = nu_lu * dx_m * dx_m / nu_phys
    e_unit = rho_phys * dx_m ** 5 / dt ** 2
    return BOLTZMANN * temp / e_unit


def capillary_units(dx_um: float, ny: int, tau: float = 1.0, Re: float = 1e-2, Ca: float = 1e-2,
                    nu_phys: float = 1.2e-6, rho_phys: float = 1000.0) -> dict:
    """Lattice values of the capillary set-up (Sec. 3) for a channel of ny
    cells of dx_um micrometres, and the scales that convert them back:
      nu       = (tau - 1/2)/3;
      u_max    = Re nu / H with H = ny (Re = u_max H / nu);
      ks       = rho nu u_max / Ca (rho = 1);
      sigma_unit = rho nu^2 / H, the unit in which sigma is given;
      y_cr     = 25 nm / dx, y_eq = y_cr / 2;
      dt_s     = nu dx^2 / nu_phys (seconds per step);
      velocity_scale = dx / dt (m/s per lattice velocity);
      stiffness_scale = rho_phys dx^3 / dt^2 (N/m per lattice spring
      constant, a 2D membrane of depth dx)."""
    nu = viscosity(tau)
    dx_m = dx_um * 1e-6
    u_max = Re * nu / ny
    dt_s = nu * dx_m * dx_m / nu_phys
    y_cr = 0.025 / dx_um
    return {"nu": nu, "u_max": u_max, "ks": nu * u_max / Ca, "sigma_unit": nu * nu / ny,
            "y_cr": y_cr, "y_eq": 0.5 * y_cr, "dx_m": dx_m, "dt_s": dt_s,
            "velocity_scale": dx_m / dt_s, "stiffness_scale": rho_phys * dx_m ** 3 / dt_s ** 2}


def poiseuille_init(nx: int, ny: int, g: float, tau: float):
    prof = poiseuille_profile(g, ny, tau)
    u0 = np.zeros((2, ny, nx))
    u0[0] = prof[:, None]
    return np.ones((ny, nx)), u0


def uniform_receptors(nx: int) -> List[np.ndarray]:
    """One receptor per wall node on each wall (positions x = 0..nx-1)."""
    x = np.arange(nx, dtype=np.float64)
    return [x.copy(), x.copy()]


# ---------------------------------------------------------------- configs

def channel_256x64(seed_offset: int = 1, with_particle: bool = True) -> Workload:
    """256x64 channel, tau = 1, Poiseuille at Mach 0.05; one RBC (120 markers)
    and one rigid 1 um particle (40 markers); constants from a seed."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))
    nx, ny, tau = 256, 64, 1.0
    u_max = 0.05 / np.sqrt(3.0)
    g = poiseuille_force(u_max, ny, tau)
    um_per_dx = 10.0 / ny                       # channel height 10 um
    alpha = 3.5 / um_per_dx                     # 22.4
    r_p = 0.5 / um_per_dx                       # 3.2
    rbc0 = geometry.rbc_contour(alpha, 120)
    ang = rng.uniform(-np.pi, np.pi)
    c = np.array([rng.uniform(48, 80), rng.uniform(24, 40)])
    rbc = geometry.place(rbc0, ang, c)
    ks = rng.uniform(5e-3, 5e-2)
    kb = rng.uniform(0.0, 5e-3)
    bodies = [Body(RBC_KINEMATIC, rbc, ks=ks, kb=kb)]
    if with_particle:
        occ = geometry.Occupancy(nx, ny)
        assert occ.try_add(rbc, 2.0)
        p0 = geometry.circle(r_p, 40)
        for _ in range(10000):
            pc = np.array([rng.uniform(0, nx), rng.uniform(6 + r_p, ny - 7 - r_p)])
            part = geometry.place(p0, 0.0, pc)
            if occ.try_add(part, 6.0):
                break
        else:
            raise RuntimeError("particle placement failed")
        bodies.append(Body(PARTICLE_RIGID, part, ks=0.0, kb=0.0))
    rho0, u0 = poiseuille_init(nx, ny, g, tau)
    return Workload("channel-256x64", nx, ny, tau, gx=g, seed=SEED_BASE + seed_offset,
                    bodies=bodies, rho0=rho0, u0=u0, steps=1000, dtype="f64")


def _capillary(name: str, nx: int, ny: int, dx_um: float, n_rbc: int, rbc_markers: int,
               particles, seed: int, steps: int, sigma_phys: float = 1.0,
               place_res: float = 1.0) -> Workload:
    """Capillary of height 10 um at Re = 0.01 with RBCs and adhesive particles.

    particles: list of (kind, sigma_phys) for 1 um carriers.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    tau = 1.0
    un = capillary_units(dx_um, ny, tau)      # Re = 1e-2, Ca = 1e-2
    nu, u_max = un["nu"], un["u_max"]
    g = poiseuille_force(u_max, ny, tau)
    alpha = 3.5 / dx_um
    r_p = 0.5 / dx_um
    ks = un["ks"]
    sig_unit = un["sigma_unit"]               # rho nu^2 / H
    y_cr = un["y_cr"]
    occ = geometry.Occupancy(nx, ny, res=place_res)
    bodies: List[Body] = []
    rbc0 = geometry.rbc_contour(alpha, rbc_markers)
    placed = 0
    tries = 0
    while placed < n_rbc:
        tries += 1
        if tries > 200000:
            raise RuntimeError("RBC placement failed")
        ang = rng.uniform(-0.25 * np.pi, 0.25 * np.pi)
        c = np.array([rng.uniform(0, nx), rng.uniform(0.0, ny)])
        xy = geometry.place(rbc0, ang, c)
        if occ.try_add(xy, 2.0):
            bodies.append(Body(RBC_KINEMATIC, xy, ks=ks, kb=0.0))
            placed += 1
    n_p = max(16, int(round(2 * np.pi * r_p / 1.0)))
    n_p += n_p % 2
    p0 = geometry.circle(r_p, n_p)
    for kind, sig in particles:
        for _ in range(200000):
            c = np.array([rng.uniform(0, nx), rng.uniform(0.0, ny)])
            xy = geometry.place(p0, rng.uniform(0, 2 * np.pi), c)
            if occ.try_add(xy, 2.0):
                break
        else:
            raise RuntimeError("particle placement failed")
        if kind == PARTICLE_RIGID:
            bodies.append(Body(PARTICLE_RIGID, xy, sigma=sig * sig_unit, ligand_stride=2))
        else:
            bodies.append(Body(PARTICLE_SOFT, xy, ks=ks, kb=0.05 * ks * r_p * r_p,
                               sigma=sig * sig_unit, ligand_stride=2))
    adh = Adhesion(y_cr=y_cr, y_eq=un["y_eq"], kf0_dt=1e-3, kr0_dt=1e-3 / 8.5e3,
                   sigma_ts_frac=0.5, kbt=kbt_lattice(dx_um * 1e-6, nu))
    rho0, u0 = poiseuille_init(nx, ny, g, tau)
    return Workload(name, nx, ny, tau, gx=g, seed=seed, bodies=bodies,
                    receptors=uniform_receptors(nx), adhesion=adh, rho0=rho0, u0=u0,
                    steps=steps, dtype="f32")


def capillary_2000x200() -> Workload:
    """10 um x 100 um capillary at dx = 50 nm (200 x 2000), 20 % hematocrit as
    18 RBCs (352 markers), 12 adhesive 1 um particles (6 rigid, 6 Ca = 1e-2),
    receptors on every wall node, sigma = 1."""
    parts = [(PARTICLE_RIGID, 1.0)] * 6 + [(PARTICLE_SOFT, 1.0)] * 6
    return _capillary("capillary-2000x200", 2000, 200, 0.05, 18, 352, parts,
                      SEED_BASE + 2, 100000)


def capillary_6667x667(soft: bool = False) -> Workload:
    """10 um x 100 um capillary at dx = 15 nm (6667 x 667), 18 RBCs (1152 markers),
    three 1 um particles with sigma = 0.5, 1, 2."""
    kind = PARTICLE_SOFT if soft else PARTICLE_RIGID
    parts = [(kind, 0.5), (kind, 1.0), (kind, 2.0)]
    return _capillary("capillary-6667x667", 6667, 667, 0.015, 18, 1152, parts,
                      SEED_BASE + 3, 50000, place_res=4.0)


def couette_box(kind: int = PARTICLE_RIGID, sigma_phys: float = 1.0, nx: int = 600,
                ny: int = 200, dx_um: float = 0.015, seed_offset: int = 6) -> Workload:
    """The paper's adhesion box: a slice of the cell-free layer next to the
    vessel wall (600 x 200 nodes at dx = 15 nm, 9 um x 3 um) between Zou-He
    velocity walls on the node rows 0 and ny - 1, the top wall moving so that
    the shear rate is the wall shear rate 4 u_max / H of the Re = 0.01
    capillary (u_max = Re nu / H, H = 10 um); one 1 um particle (rigid, or
    soft with Ca = 1e-2 and E_b = 0.05) released with its lowest vertex at the
    bond rest length y_eq above the lower wall, ligands on every other
    element, receptors on every wall node; sigma in units rho nu^2 / H."""
    tau = 1.0
    nu = viscosity(tau)
    h_cap = 10.0 / dx_um
    u_max = 0.01 * nu / h_cap
    u_top = 4.0 * u_max / h_cap * (ny - 1)
    r_p = 0.5 / dx_um
    ks = nu * u_max / 1e-2
    sig_unit = nu * nu / h_cap
    y_cr = 0.025 / dx_um
    n_p = max(16, int(round(2 * np.pi * r_p / 1.0)))
    n_p += n_p % 2
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))
    xy = geometry.place(geometry.circle(r_p, n_p), rng.uniform(0, 2 * np.pi),
                        [0.25 * nx, 0.0])
    xy[:, 1] += 0.5 * y_cr - xy[:, 1].min()
    if kind == PARTICLE_RIGID:
        body = Body(PARTICLE_RIGID, xy, sigma=sigma_phys * sig_unit, ligand_stride=2)
    else:
        body = Body(PARTICLE_SOFT, xy, ks=ks, kb=0.05 * ks * r_p * r_p,
                    sigma=sigma_phys * sig_unit, ligand_stride=2)
    adh = Adhesion(y_cr=y_cr, y_eq=0.5 * y_cr, kf0_dt=1e-3, kr0_dt=1e-3 / 8.5e3,
                   sigma_ts_frac=0.5, kbt=kbt_lattice(dx_um * 1e-6, nu))
    y = np.arange(ny, dtype=np.float64)
    u0 = np.zeros((2, ny, nx))
    u0[0] = (u_top * y / (ny - 1))[:, None]
    name = f"couette-box-{nx}x{ny}-{'rigid' if kind == PARTICLE_RIGID else 'soft'}-sigma{sigma_phys:g}"
    return Workload(name, nx, ny, tau, seed=SEED_BASE + seed_offset, bodies=[body],
                    receptors=uniform_receptors(nx), adhesion=adh, u0=u0,
                    walls="zou-he", u_wall=(0.0, u_top), steps=20000, dtype="f32")


def sweep_instances(n_inst: int = 64, seed_offset: int = 4) -> List[Workload]:
    """Uneven capillary instances (20-100 um long, dx = 50 nm, 200 rows),
    20 % hematocrit, four particles each; (Ca, sigma) cycle over
    {0, 1e-2} x {0.5, 1, 2}."""
    out = []
    combos = [(k, s) for k in (PARTICLE_RIGID, PARTICLE_SOFT) for s in (0.5, 1.0, 2.0)]
    lrng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))
    lengths = lrng.uniform(20.0, 100.0, size=n_inst)
    for i in range(n_inst):
        L = float(lengths[i])
        nx = int(round(L / 0.05))
        n_rbc = int(round(0.2 * 10.0 * L / 10.92))
        kind, sig = combos[i % len(combos)]
        w = _capillary(f"sweep-inst{i}", nx, 200, 0.05, n_rbc, 352, [(kind, sig)] * 4,
                       SEED_BASE + seed_offset + i, 20000)
        w.instance = i
        w.seed = SEED_BASE + seed_offset
        out.append(w)
    return out


def adjoint_channel(nx: int = 256, ny: int = 64, seed_offset: int = 5, ks_particle: float = 0.02,
                    sigma: float = 1e-3, n_rbc: int = 1, rigid: bool = False) -> Workload:
    """Gradient window: the 256x64 channel with its seeded red cell, and the
    1 um particle made soft (k_s = 0.02, E_b = 0.05; or rigid) and released
    next to the lower wall with its lowest vertex at a wall distance of
    y_cr / 2, so that bonds form at the first step.  Adhesion in lattice
    units: y_cr = 0.5, y_eq = 0.25, sigma = 1e-3, k_f0 dt = 0.5 (bonds form at
    once)."""
    base = channel_256x64(seed_offset=1, with_particle=False)
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))
    scale = ny / base.ny
    g = poiseuille_force(0.05 / np.sqrt(3.0), ny, base.tau)
    bodies: List[Body] = []
    if n_rbc:
        rbc = base.bodies[0]
        xy = rbc.xy * scale
        bodies.append(Body(RBC_KINEMATIC, xy, ks=rbc.ks, kb=rbc.kb))
    r_p = 0.5 / (10.0 / ny)
    p0 = geometry.circle(r_p, 40)
    y_cr = 0.5
    x_c = float(bodies[0].xy[:, 0].mean() + 0.5 * nx) if bodies else rng.uniform(0, nx)
    y_c = -0.5 + 0.5 * y_cr - p0[:, 1].min()
    xy = geometry.place(p0, 0.0, [x_c % nx, y_c])
    if rigid:
        bodies.append(Body(PARTICLE_RIGID, xy, sigma=sigma, ligand_stride=2))
    else:
        bodies.append(Body(PARTICLE_SOFT, xy, ks=ks_particle, kb=0.05 * ks_particle * r_p * r_p,
                           sigma=sigma, ligand_stride=2))
    rho0, u0 = poiseuille_init(nx, ny, g, base.tau)
    adh = Adhesion(y_cr=y_cr, y_eq=0.5 * y_cr, kf0_dt=0.5, kr0_dt=0.5 / 8.5e3,
                   sigma_ts_frac=0.5, kbt=1e-3)
    return Workload(f"adjoint-channel-{nx}x{ny}" + ("-rigid" if rigid else ""), nx, ny, base.tau, gx=g,
                    seed=SEED_BASE + seed_offset, bodies=bodies,
                    receptors=uniform_receptors(nx), adhesion=adh, rho0=rho0, u0=u0,
                    steps=2000, dtype="f32")


def small_case(nx: int = 48, ny: int = 24, seed_offset: int = 11, n_rbc: int = 1,
               particles=(), adhesive: bool = False, tau: float = 1.0,
               periodic_y: int = 0, mach: float = 0.05) -> Workload:
    """Small seeded case for parity tests: spans several 64x4 tiles only in
    larger instances; bodies scaled to the channel."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))
    u_max = mach / np.sqrt(3.0)
    g = 0.0 if periodic_y else poiseuille_force(u_max, ny, tau)
    occ = geometry.Occupancy(nx, ny)
    bodies: List[Body] = []
    alpha = 0.3 * ny
    for _ in range(n_rbc):
        nv = int(max(24, 2 * np.ceil(2.5 * alpha)))
        rbc0 = geometry.rbc_contour(alpha, nv)
        for _ in range(100000):
            xy = geometry.place(rbc0, rng.uniform(-0.3, 0.3),
                                [rng.uniform(0, nx), rng.uniform(0, ny)])
            if occ.try_add(xy, 2.0):
                break
        else:
            raise RuntimeError("placement failed")
        bodies.append(Body(RBC_KINEMATIC, xy, ks=rng.uniform(5e-3, 5e-2),
                           kb=rng.uniform(0, 5e-3)))
    r_p = max(2.5, 0.08 * ny)
    for kind in particles:
        p0 = geometry.circle(r_p, 24)
        for _ in range(100000):
            xy = geometry.place(p0, rng.uniform(0, 2 * np.pi),
                                [rng.uniform(0, nx), rng.uniform(0, ny)])
            if occ.try_add(xy, 2.0):
                break
        else:
            raise RuntimeError("placement failed")
        if kind == PARTICLE_RIGID:
            bodies.append(Body(PARTICLE_RIGID, xy, sigma=5e-3 if adhesive else 0.0,
                               ligand_stride=2 if adhesive else 0))
        else:
            ks = 2e-2
            bodies.append(Body(PARTICLE_SOFT, xy, ks=ks, kb=0.05 * ks * r_p * r_p,
                               sigma=5e-3 if adhesive else 0.0,
                               ligand_stride=2 if adhesive else 0))
    if periodic_y:
        rho0, u0 = np.ones((ny, nx)), np.zeros((2, ny, nx))
    else:
        rho0, u0 = poiseuille_init(nx, ny, g, tau)
    adh = Adhesion(y_cr=1.0, y_eq=0.5, kf0_dt=0.2, kr0_dt=0.01, sigma_ts_frac=0.5, kbt=1e-3)
    return Workload(f"small-{nx}x{ny}", nx, ny, tau, gx=g, periodic_y=periodic_y,
                    seed=SEED_BASE + seed_offset, bodies=bodies,
                    receptors=uniform_receptors(nx) if adhesive else [np.zeros(0), np.zeros(0)],
                    adhesion=adh, rho0=rho0, u0=u0, steps=200)
