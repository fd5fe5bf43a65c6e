"""Pins of the lattice-unit conversions of the capillary set-up (Sec. 3)
against the physical values the paper prints: the channel of H = 10 um
discretised with 200 cells (dx = 50 nm), water viscosity 1.2e-6 m^2/s,
Re = 1e-2 giving a centre-line velocity of 1.2e-3 m/s, Ca = 1e-2 with a
membrane stiffness quoted as 1.5e-4 N/m, y_cr = 25 nm with y_eq = y_cr / 2,
sigma in units of rho nu^2 / H, particle to fluid density ratio 1.1."""
import numpy as np
import pytest

from workloads import configs


def test_centre_line_velocity_converts_to_the_printed_value():
    u = configs.capillary_units(0.05, 200)
    assert abs(u["u_max"] * 200 / u["nu"] - 1e-2) < 1e-15          # Re in lattice units
    assert abs(u["u_max"] * u["velocity_scale"] - 1.2e-3) < 1e-15    # m/s, Sec. 3
    assert abs(u["dt_s"] - (1 / 6) * (5e-8) ** 2 / 1.2e-6) < 1e-24   # 3.47e-10 s


@pytest.mark.parametrize("dx_um, ny", [(0.05, 200), (0.015, 667)])
def test_membrane_stiffness_matches_the_quoted_value(dx_um, ny):
    """k_s = rho nu u_max / Ca in lattice units, converted to N/m, equals the same
    formula in SI units (1.44e-4 N/m at 200 cells) and lies within 4.5 % of the
    1.5e-4 N/m the paper quotes for Ca = 1e-2 (the quoted value is that product
    rounded to two digits)."""
    u = configs.capillary_units(dx_um, ny)
    ks_si = u["ks"] * u["stiffness_scale"]
    H = dx_um * 1e-6 * ny
    u_si = 1e-2 * 1.2e-6 / H
    assert abs(ks_si / (1000.0 * 1.2e-6 * u_si / 1e-2) - 1.0) < 1e-12
    assert abs(ks_si / 1.5e-4 - 1.0) < 0.045


def test_bond_constants_in_lattice_units():
    u50 = configs.capillary_units(0.05, 200)
    assert abs(u50["y_cr"] - 0.5) < 1e-15 and u50["y_eq"] == 0.5 * u50["y_cr"]
    assert abs(configs.capillary_units(0.015, 667)["y_cr"] - 25 / 15) < 1e-15
    # sigma = 1 in units rho nu^2 / H: (1/36)/200 in lattice units, and the
    # same unit converted to N/m equals rho nu^2 / H in SI
    assert abs(u50["sigma_unit"] - (1 / 36) / 200) < 1e-18
    si = u50["sigma_unit"] * u50["stiffness_scale"]
    assert abs(si / (1000.0 * 1.2e-6 ** 2 / 10e-6) - 1.0) < 1e-12


def test_capillary_workloads_carry_the_converted_constants():
    wl = configs.capillary_2000x200()
    u = configs.capillary_units(0.05, 200)
    rbc = [b for b in wl.bodies if b.kind == configs.RBC_KINEMATIC]
    parts = [b for b in wl.bodies if b.kind != configs.RBC_KINEMATIC]
    assert len(rbc) == 18 and len(parts) == 12
    assert all(b.ks == u["ks"] and b.kb == 0.0 for b in rbc)
    assert all(abs(b.sigma - u["sigma_unit"]) < 1e-18 and b.density_ratio == 1.1 for b in parts)
    soft = [b for b in parts if b.kind == configs.PARTICLE_SOFT]
    r_p = 0.5 / 0.05
    assert all(abs(b.kb - 0.05 * b.ks * r_p ** 2) < 1e-18 for b in soft)    # E_b = 0.05
    assert wl.adhesion.y_cr == u["y_cr"] and wl.adhesion.y_eq == u["y_eq"]
    assert abs(wl.adhesion.kf0_dt / wl.adhesion.kr0_dt - 8.5e3) < 1e-9
    # the drive gives the discrete steady profile its centre-line speed u_max
    prof = configs.poiseuille_profile(wl.gx, wl.ny, wl.tau)
    assert abs(prof.max() / u["u_max"] - 1.0) < 1e-3
