"""Pins of the observables oracle (Sec. 3 quantities) against closed forms:
the centre of a regular polygon, the region boundaries of the paper, and a
scripted sequence of displacements with known maxima and velocities."""
import numpy as np
import pytest

from oracle import observables as obs


def polygon(n, r, cx, cy, phase=0.3):
    a = phase + 2.0 * np.pi * np.arange(n) / n
    return np.stack([cx + r * np.cos(a), cy + r * np.sin(a)], axis=1)


def test_centre_of_regular_polygon():
    c = obs.centre_of_mass(polygon(24, 3.0, 17.25, 8.5))
    assert c == pytest.approx([17.25, 8.5], abs=1e-13)


@pytest.mark.parametrize("eta, reg", [(0.05, obs.CFL), (0.2, obs.CFL), (0.2000001, obs.INTERMEDIATE),
                                      (0.25, obs.INTERMEDIATE), (0.3, obs.BULK), (0.5, obs.BULK),
                                      (0.7, obs.BULK), (0.75, obs.INTERMEDIATE),
                                      (0.8, obs.CFL), (0.95, obs.CFL)])
def test_regions_of_the_paper(eta, reg):
    ny = 200
    yc = eta * ny - 0.5           # eta = (y + 1/2) / H with walls at -1/2 and ny - 1/2
    assert obs.region(yc, ny) == reg


def test_scripted_trajectory():
    ny = 100
    base = polygon(16, 2.0, 10.0, 30.0)
    o = obs.Observer(1)
    # (step, shift x, shift y, bonds): displacements chosen by hand
    script = [(0, 0.0, 0.0, 2), (10, 1.0, 4.0, 3), (30, 5.0, -6.0, 0), (35, 6.0, -1.0, 1)]
    for step, sx, sy, nb in script:
        o.observe(step, [base + [sx, sy]], [nb], ny)
    r = o.obs[0]
    assert (r.x0, r.y0) == pytest.approx((10.0, 30.0), abs=1e-13)
    assert r.r_max == pytest.approx(6.0, abs=1e-13)       # the largest |dy| was at step 30
    assert r.u_x == pytest.approx(1.0 / 5.0, abs=1e-13)    # last interval: dx 1 over 5 steps
    assert r.u_y == pytest.approx(5.0 / 5.0, abs=1e-13)
    assert r.u_x_sum == pytest.approx(1.0 / 10 + 4.0 / 20 + 1.0 / 5, abs=1e-13)
    assert r.u_y_sum == pytest.approx(4.0 / 10 - 10.0 / 20 + 5.0 / 5, abs=1e-13)
    assert (r.n_bonds, r.n_bonds0, r.n_obs, r.step_obs) == (1, 2, 4, 35)
    assert r.region == obs.region(29.0, ny) == obs.INTERMEDIATE    # eta = 29.5 / 100 = 0.295


def test_observer_of_a_sim_counts_bonds_per_body():
    from workloads import configs
    from oracle import sim as osim
    xy = polygon(12, 3.0, 20.0, 3.0)
    wl = configs.Workload("o", 48, 24, bodies=[
        configs.Body(configs.PARTICLE_RIGID, xy, ligand_stride=2),
        configs.Body(configs.PARTICLE_RIGID, polygon(12, 3.0, 35.0, 12.0), ligand_stride=3)])
    s = osim.Sim(wl)
    s.l2r[:] = -1
    s.l2r[[0, 2, 7]] = 0          # ligands 0, 2 (body 0) and 7 (body 1: body 0 has 6)
    o = obs.Observer(2)
    o.observe_sim(s)
    assert [r.n_bonds for r in o.obs] == [2, 1]
    assert o.obs[0].region == obs.CFL and o.obs[1].region == obs.BULK
