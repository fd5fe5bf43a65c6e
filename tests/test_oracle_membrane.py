"""Pins of the oracle's membrane forces (Sec. 2.2, Eqs. strainFor, bendFor, areaFor)."""
import os

import numpy as np
import pytest

from oracle import membrane
from workloads import geometry


def _shapes():
    rbc = geometry.place(geometry.rbc_contour(22.4, 120), 0.7, [50.0, 30.0])
    circ = geometry.place(geometry.circle(3.2, 40), 0.0, [10.0, 8.0])
    return [rbc, circ]


@pytest.mark.parametrize("k", [0, 1])
def test_zero_force_at_rest_shape(k):
    xy = _shapes()[k]
    l0, _, _ = membrane.elements(xy)
    th0 = membrane.turning_angles(xy)
    A0 = membrane.area(xy)
    F = membrane.internal_force(xy, l0, th0, A0, 0.03, 0.004, 1.0, 1 / 3)
    assert np.max(np.abs(F)) < 1e-15


def test_area_matches_exact_polygons():
    # unit square, and the area of a regular n-gon n r^2 sin(2 pi/n)/2
    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    assert membrane.area(sq) == 1.0
    for n in (6, 40, 128):
        c = geometry.circle(2.5, n)
        assert abs(membrane.area(c) - 0.5 * n * 2.5 ** 2 * np.sin(2 * np.pi / n)) < 1e-12
    assert membrane.area(sq[::-1]) == -1.0


def test_turning_angles_regular_polygon():
    for n in (5, 12, 40):
        th = membrane.turning_angles(geometry.circle(1.7, n))
        assert np.allclose(th, 2 * np.pi / n, atol=1e-14)
        assert abs(th.sum() - 2 * np.pi) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forces_sum_to_zero_and_strain_is_gradient(seed):
    rng = np.random.default_rng(seed)
    xy0 = _shapes()[seed % 2]
    l0, _, _ = membrane.elements(xy0)
    th0 = membrane.turning_angles(xy0)
    A0 = membrane.area(xy0)
    xy = xy0 + 0.2 * rng.standard_normal(xy0.shape)
    ks, kb = 0.02, 0.003
    Fs = membrane.strain_force(xy, l0, ks)
    Fb = membrane.bending_force(xy, th0, kb)
    Fa = membrane.area_force(xy, A0, 1.0, 1 / 3)
    for F in (Fs, Fb, Fa):
        assert np.max(np.abs(F.sum(0))) < 1e-14
    # strain force is central: no net torque
    assert abs(np.sum(xy[:, 0] * Fs[:, 1] - xy[:, 1] * Fs[:, 0])) < 1e-12
    # strain force = -grad of V = ks (l - l0)^2 / 2 (Eq. strainPot), central differences
    h = 1e-6
    G = np.zeros_like(xy)
    for v in range(xy.shape[0]):
        for a in range(2):
            p, m = xy.copy(), xy.copy()
            p[v, a] += h
            m[v, a] -= h
            G[v, a] = (membrane.strain_energy(p, l0, ks) - membrane.strain_energy(m, l0, ks)) / (2 * h)
    assert np.max(np.abs(Fs + G)) < 1e-8 * max(1.0, np.max(np.abs(Fs)))


def test_area_force_on_scaled_circle_is_radial_closed_form():
    n, r, s = 48, 4.0, 0.9
    xy0 = geometry.circle(r, n)
    A0 = membrane.area(xy0)
    xy = s * xy0
    ka, pref = 1.0, 1 / 3
    F = membrane.area_force(xy, A0, ka, pref)
    # each element: ka (1 - s^2) pref l n, l = 2 s r sin(pi/n); vertex gets two halves
    # whose sum is radial with magnitude ka (1 - s^2) pref l cos(pi/n)
    l = 2 * s * r * np.sin(np.pi / n)
    mag = ka * (1 - s * s) * pref * l * np.cos(np.pi / n)
    rad = xy / np.hypot(xy[:, 0], xy[:, 1])[:, None]
    assert np.allclose(F, mag * rad, atol=1e-14)


def test_bending_restoring_direction():
    n = 24
    xy0 = geometry.circle(5.0, n)
    th0 = membrane.turning_angles(xy0)
    xy = xy0.copy()
    xy[3] *= 1.05       # push vertex 3 outward -> sharper corner -> inward force on it
    F = membrane.bending_force(xy, th0, 1.0)
    rad = xy[3] / np.linalg.norm(xy[3])
    assert F[3] @ rad < 0
    # only the perturbed vertex and its neighbours' angles change: forces confined to v=1..5
    nz = np.nonzero(np.abs(F).sum(1) > 1e-14)[0]
    assert set(nz) <= {1, 2, 3, 4, 5}
    # bending is invariant to scaling and rotation of the rest shape
    F2 = membrane.bending_force(geometry.place(2.0 * xy0, 0.4, [3, 3]), th0, 1.0)
    assert np.max(np.abs(F2)) < 1e-13


def _golden_bending():
    rows, kb = [], None
    with open(os.path.join(os.path.dirname(__file__), "golden", "bending_rectangle_4x1.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            vals = [float(v) for v in line.split()]
            if kb is None:
                kb = vals[0]
            else:
                rows.append(vals)
    a = np.array(rows)
    return kb, a[:, 1:3], a[:, 3], a[:, 4:6]


def test_bending_hand_worked_rectangle():
    """Eq. bendFor worked by hand on a 4 x 1 rectangle bent at one corner whose
    two edges differ in length (fixture and derivation in tests/golden/)."""
    kb, xy, th0, F_expected = _golden_bending()
    F = membrane.bending_force(xy, th0, kb)
    assert np.max(np.abs(F - F_expected)) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_internal_forces_exert_no_net_moment(seed):
    """Internal membrane forces cannot change the body's angular momentum: the
    bending triple of every vertex (with unequal edge lengths), the central
    strain pairs and the area loads all have zero moment about any point."""
    rng = np.random.default_rng(100 + seed)
    xy0 = _shapes()[seed % 2]
    l0, _, _ = membrane.elements(xy0)
    th0 = membrane.turning_angles(xy0)
    A0 = membrane.area(xy0)
    # strongly uneven vertex spacing: element lengths differ by up to 3x
    xy = xy0 + 0.25 * rng.standard_normal(xy0.shape)
    length, _, _ = membrane.elements(xy)
    assert length.max() / length.min() > 3.0
    ref = rng.uniform(-20, 20, size=2)
    for F in (membrane.bending_force(xy, th0, 0.01), membrane.strain_force(xy, l0, 0.02),
              membrane.area_force(xy, A0, 1.0, 1 / 3)):
        r = xy - ref[None, :]
        M = np.sum(r[:, 0] * F[:, 1] - r[:, 1] * F[:, 0])
        scale = np.sum(np.hypot(r[:, 0], r[:, 1]) * np.hypot(F[:, 0], F[:, 1]))
        assert abs(M) < 1e-13 * scale
        assert np.max(np.abs(F.sum(0))) < 1e-13 * np.max(np.abs(F))
