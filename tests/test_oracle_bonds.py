"""Pins of the oracle's adhesion model (Sec. 2.2 Wall-Particle Interaction, Eq. adhFor).

Philox is pinned to the published known-answer vectors; the deterministic
limit of the kinetics (certain formation, no rupture) is checked against
the properties that define greedy nearest-free matching, written
independently; the stochastic case against binomial confidence bounds;
the spring law against its closed form.
"""
import math
import os

import numpy as np
import pytest

from oracle import adhesion, philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert philox.philox4x32_10(ctr, key) == out


def test_philox_uniformity_chi2():
    counts = np.zeros(16)
    N = 8000
    for l in range(N):
        u = philox.uniform(12345, 7, l, 0)
        assert 0.0 <= u < 1.0
        counts[int(u * 16)] += 1
    chi2 = ((counts - N / 16) ** 2 / (N / 16)).sum()
    assert chi2 < 37.7  # 15 dof, p = 0.001


def _params(**kw):
    p = dict(y_cr=1.0, y_eq=0.5, kf0_dt=1e3, kr0_dt=0.0, sigma_ts_frac=0.5, kbt=1e30)
    p.update(kw)
    return adhesion.BondParams(**p)


@pytest.mark.parametrize("seed", range(6))
def test_deterministic_limit_is_greedy_matching(seed):
    """k_f0 dt huge and k_r0 = 0: every eligible ligand bonds to its nearest
    free receptor, taken in ascending ligand order."""
    rng = np.random.default_rng(seed)
    nx, ny = 12, 10
    nl = 9
    c = np.stack([rng.uniform(-3, nx + 3, nl), rng.choice([0.1, 0.3, ny - 1.2, ny - 1.4, 5.0], nl)], 1)
    rec = [np.sort(rng.choice(nx, 4, replace=False)).astype(float),
           np.sort(rng.choice(nx, 3, replace=False)).astype(float)]
    p = _params()
    l2r, ties = adhesion.bond_update(0, c, np.ones(nl), -np.ones(nl, int), rec, nx, ny, p, seed)
    assert ties == 0
    n0 = len(rec[0])
    taken = [r for r in l2r if r >= 0]
    assert len(taken) == len(set(taken))               # one bond per receptor

    def wall_of(cy):
        return 0 if (cy + 0.5) <= (ny - 0.5 - cy) else 1

    def dist(l, xr):
        d = abs(((xr - (c[l, 0] % nx)) + nx / 2) % nx - nx / 2)
        return d

    for l in range(nl):
        w = wall_of(c[l, 1])
        dwall = min(c[l, 1] + 0.5, ny - 0.5 - c[l, 1])
        ids = range(n0) if w == 0 else range(n0, n0 + len(rec[1]))
        xs = rec[0] if w == 0 else rec[1]
        if dwall >= p.y_cr:
            assert l2r[l] == -1
            continue
        # receptors still free when ligand l was considered: not taken by lower ids
        before = {l2r[k] for k in range(l) if l2r[k] >= 0}
        avail = [r for r in ids if r not in before]
        if not avail:
            assert l2r[l] == -1
            continue
        assert l2r[l] in avail
        dmin = min(dist(l, xs[r - (0 if w == 0 else n0)]) for r in avail)
        chosen = l2r[l] - (0 if w == 0 else n0)
        assert abs(dist(l, xs[chosen]) - dmin) < 1e-12
        # ties go to the lower receptor index
        assert l2r[l] == min(r for r in avail
                             if abs(dist(l, xs[r - (0 if w == 0 else n0)]) - dmin) < 1e-12)


def test_rupture_certain_and_no_reforming_in_same_step():
    nx, ny = 8, 6
    c = np.array([[2.2, 0.1], [5.0, 0.2]])
    rec = [np.arange(nx, dtype=float), np.arange(nx, dtype=float)]
    p = _params(kr0_dt=1e6)
    l2r, _ = adhesion.bond_update(3, c, np.ones(2), np.array([2, 5]), rec, nx, ny, p, 1)
    assert (l2r == -1).all()                           # ruptured, cannot re-form this step
    l2r, _ = adhesion.bond_update(4, c, np.ones(2), l2r, rec, nx, ny, _params(), 1)
    assert list(l2r) == [2, 5]                          # nearest receptors, next step


def test_formation_frequency_matches_probability():
    nx, ny = 16, 8
    p = _params(kf0_dt=0.3, sigma_ts_frac=0.0, kbt=1.0)
    P = 1 - math.exp(-0.3)                              # sigma_ts = 0: k_f = k_f0
    assert abs(adhesion.formation_probability(0.37, 2.0, p) - P) < 1e-15
    c = np.array([[4.3, 0.2]])
    rec = [np.arange(nx, dtype=float), np.arange(nx, dtype=float)]
    N = 3000
    hits = 0
    for step in range(N):
        l2r, _ = adhesion.bond_update(step, c, np.ones(1), -np.ones(1, int), rec, nx, ny, p, 99)
        hits += l2r[0] >= 0
    sd = math.sqrt(N * P * (1 - P))
    assert abs(hits - N * P) < 5 * sd


def test_rates_closed_form():
    p = adhesion.BondParams(y_cr=1.0, y_eq=0.5, kf0_dt=0.01, kr0_dt=0.002, sigma_ts_frac=0.25, kbt=0.1)
    y, sig = 0.9, 0.4
    kf = 0.01 * math.exp(-0.1 * 0.16 / 0.2)
    kr = 0.002 * math.exp(0.3 * 0.16 / 0.2)
    assert abs(adhesion.formation_probability(y, sig, p) - (1 - math.exp(-kf))) < 1e-16
    assert abs(adhesion.rupture_probability(y, sig, p) - (1 - math.exp(-kr))) < 1e-16


def test_spring_zero_at_equilibrium_and_linear():
    nx, ny = 10, 8
    n = np.array([0.0, -1.0])
    y_eq = 0.25
    # centroid straight above receptor at x = 3 on wall 0 (y = -1/2)
    for d, expect in [(0.25, 0.0), (0.75, 0.5), (1.25, 1.0)]:
        c = np.array([3.0, -0.5 + d])
        F = adhesion.spring_force(c, n, 3.0, 0, 2.0, y_eq, nx, ny)
        assert np.allclose(F, 2.0 * (d - y_eq) * n, atol=1e-15)
        assert abs(np.linalg.norm(F) - 2.0 * expect) < 1e-15
    # minimum image across the periodic seam
    c = np.array([9.8, -0.5 + 0.3])
    F = adhesion.spring_force(c, n, 0.2, 0, 1.0, y_eq, nx, ny)
    assert abs(np.linalg.norm(F) - (math.hypot(0.4, 0.3) - y_eq)) < 1e-14
