"""Pins of the repulsion oracle (Sec. 2.2, Eq. repFor) against closed forms,
cut-off and exclusion rules, the minimum image, and the step's force and
torque bookkeeping."""
import numpy as np
import pytest

from oracle import repulsion, sim as osim
from workloads import configs

C = 8.838834764831844e-06     # 1e-4 / (8 sqrt 2)


def polygon(n, r, cx, cy, phase=0.0):
    a = phase + 2.0 * np.pi * np.arange(n) / n
    return np.stack([cx + r * np.cos(a), cy + r * np.sin(a)], axis=1)


def tip_pair(d, cx=20.0, cy=20.0):
    """Two regular octagons of radius 3 whose vertices 0 (at angle 0) and 4
    (at angle pi) face each other at distance d; their other vertices are
    more than 2 apart."""
    A = polygon(8, 3.0, cx, cy)
    B = polygon(8, 3.0, cx + 6.0 + d, cy)
    return A, B


def test_coefficient_is_the_papers():
    assert repulsion.COEFF == pytest.approx(C, rel=1e-15)


@pytest.mark.parametrize("d, dpow", [(1.0, 1.0), (0.64, 3.0517578125), (0.25, 32.0)])
def test_single_pair_closed_form(d, dpow):
    A, B = tip_pair(d)
    FA, FB = repulsion.forces([A, B], C, 2.0, 64, 64, False)
    # only the facing tips interact; each is pushed straight back into its body
    expect = C * dpow
    assert FA[0] == pytest.approx([-expect, 0.0], rel=1e-12, abs=1e-22)
    assert FB[4] == pytest.approx([expect, 0.0], rel=1e-12, abs=1e-22)
    assert np.all(FA[1:] == 0.0) and np.all(np.delete(FB, 4, axis=0) == 0.0)
    # symmetric pair: equal and opposite
    assert np.allclose(FA.sum(axis=0) + FB.sum(axis=0), 0.0, atol=1e-22)


def test_cutoff_edges():
    A, B = tip_pair(1.999)
    FA, _ = repulsion.forces([A, B], C, 2.0, 64, 64, False)
    assert FA[0, 0] < 0.0
    A, B = tip_pair(2.001)
    FA, FB = repulsion.forces([A, B], C, 2.0, 64, 64, False)
    assert np.all(FA == 0.0) and np.all(FB == 0.0)


def test_no_self_repulsion():
    # a thin rectangle: its two long sides are 1 apart, but one body
    xs = np.arange(0.0, 10.0, 1.0)
    top = np.stack([xs[::-1], np.full_like(xs, 11.0)], axis=1)
    bot = np.stack([xs, np.full_like(xs, 10.0)], axis=1)
    thin = np.concatenate([bot, top])[:, :] + np.array([10.0, 0.0])
    F, = repulsion.forces([thin], C, 2.0, 64, 64, False)
    assert np.all(F == 0.0)


def test_minimum_image_in_x_and_y():
    d = 0.8
    A, B = tip_pair(d, cx=30.0, cy=30.0)
    ref = repulsion.forces([A, B], C, 2.0, 64, 64, False)
    # shift the pair so that it straddles the x seam at 0 / nx
    nx = 64
    s = np.array([-(30.0 + 3.0 + 0.5 * d), 0.0])
    A2, B2 = np.mod(A + s, [nx, 1e9]), np.mod(B + s, [nx, 1e9])
    assert A2[0, 0] > 60.0 and B2[4, 0] < 1.0          # the tips are on opposite sides
    got = repulsion.forces([A2, B2], C, 2.0, nx, 64, False)
    for x, y in zip(got, ref):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-18)
    # the same along y on a periodic lattice (pair rotated by 90 degrees)
    rot = np.array([[0.0, -1.0], [1.0, 0.0]])
    A3 = (A - 30.0) @ rot.T + np.array([30.0, 0.0])
    B3 = (B - 30.0) @ rot.T + np.array([30.0, 0.0])
    ny = 48
    s = np.array([0.0, -(3.0 + 0.5 * d)])
    A3, B3 = np.mod(A3 + s, [1e9, ny]), np.mod(B3 + s, [1e9, ny])
    got = repulsion.forces([A3, B3], C, 2.0, 64, ny, True)
    for x, y in zip(got, ref):
        assert np.allclose(x, y @ rot.T, rtol=1e-12, atol=1e-18)
    # without y periodicity the pair across the y seam is far apart
    got = repulsion.forces([A3, B3], C, 2.0, 64, ny, False)
    assert all(np.all(x == 0.0) for x in got)


def test_permutation_and_three_bodies():
    A, B = tip_pair(0.9)
    Cc = polygon(8, 3.0, 20.0, 20.0 + 6.0 + 0.7, phase=0.0)   # above A, vertex 6 faces A's 2
    F = repulsion.forces([A, B, Cc], C, 2.0, 128, 128, False)
    G = repulsion.forces([Cc, A, B], C, 2.0, 128, 128, False)
    assert np.array_equal(F[0], G[1]) and np.array_equal(F[1], G[2]) and np.array_equal(F[2], G[0])
    # A's tip 0 feels B only; its vertex 2 (top) feels C's vertex 6
    assert F[0][2] == pytest.approx([0.0, -C * 0.7 ** -2.5], rel=1e-12, abs=1e-20)


def _pair_workload(kind_b, d):
    A, B = tip_pair(d, cx=20.0, cy=16.0)
    return configs.Workload(
        name="rep-pair", nx=48, ny=32, tau=1.0, periodic_y=0,
        bodies=[configs.Body(kind=configs.RBC_KINEMATIC, xy=A, ks=0.0, kb=0.0, ka=0.0),
                configs.Body(kind=kind_b, xy=B, ks=0.0, kb=0.0, ka=0.0)],
        repulsion=C, repulsion_cutoff=2.0)


def test_step_uses_repulsion_on_rbc_and_rigid():
    d = 0.9
    wl = _pair_workload(configs.PARTICLE_RIGID, d)
    s = osim.Sim(wl)
    s.step(1)
    # the red cell spreads only the repulsion (its membrane is force free)
    F = s.marker_force[0]
    assert F[0] == pytest.approx([-C * d ** -2.5, 0.0], rel=1e-12)
    assert np.all(F[1:] == 0.0)
    # the rigid particle: radial force at its tip -> no torque from it, and
    # its velocity gains the repulsion over its mass on top of the fluid loads
    wl0 = _pair_workload(configs.PARTICLE_RIGID, d)
    wl0.repulsion = 0.0
    s0 = osim.Sim(wl0)
    s0.step(1)
    b, b0 = s.bodies[1], s0.bodies[1]
    assert b.U[0] - b0.U[0] == pytest.approx(C * d ** -2.5 / b.mass, rel=1e-9)
    assert b.U[1] == pytest.approx(b0.U[1], abs=1e-18)
    assert b.Om == pytest.approx(b0.Om, abs=1e-18)


def test_far_bodies_unchanged():
    wl = _pair_workload(configs.PARTICLE_SOFT, 5.0)
    wl0 = _pair_workload(configs.PARTICLE_SOFT, 5.0)
    wl0.repulsion = 0.0
    a, b = osim.Sim(wl), osim.Sim(wl0)
    a.step(3)
    b.step(3)
    assert np.array_equal(a.all_markers(), b.all_markers())
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
