"""Local reverse-mode derivatives of the adjoint (host build of adj_math.h).

Each vector-Jacobian product is checked against central finite differences
of its forward formula: for random inputs x and output adjoints a,
(f(x + h e_k) - f(x - h e_k)) / (2h) . a must equal the k-th entry of the
VJP.  The Roma kernel's derivatives are checked the same way.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_00080_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "native", "adj_math_check.cpp")

D = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("adjmath") / "libadjcheck.so")
    subprocess.run([gxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, "-o", out, SRC],
                   check=True)
    L = ctypes.CDLL(out)
    for name in ("t_phi", "t_dphi", "t_ddphi"):
        getattr(L, name).restype = ctypes.c_double
        getattr(L, name).argtypes = [ctypes.c_double]
    d = ctypes.c_double
    sig = {"t_collide_fwd": [D, d, d, d, d, D], "t_collide_vjp": [D, d, d, d, d, D, d, d, D],
           "t_star_vjp": [d, d, d, d, d, d, D], "t_strain_fwd": [d, d, d, d, D],
           "t_strain_vjp": [d, d, d, d, d, d, D], "t_bend_fwd": [D, d, d, D],
           "t_bend_vjp": [D, d, d, D, D], "t_spring_vjp": [d, d, d, d, d, d, d, d, d, D],
           "t_hydro_fwd": [d, D, d, d, d, d, D], "t_hydro_vjp": [d, D, d, d, d, d, d, d, D],
           "t_area_vjp": [d, d, d, d, d, D], "t_spring_fwd": [d, d, d, d, d, D],
           "t_rigid_load_vjp": [d, d, d, d, d, d, d, D], "t_rigid_vertex_fwd": [d, d, D, D],
           "t_rigid_vertex_vjp": [d, d, d, D, D, D]}
    for name, args in sig.items():
        getattr(L, name).argtypes = args
        getattr(L, name).restype = None
    L.t_bdf2_vjp.argtypes = [ctypes.c_int, d, d, D]
    L.t_bdf2_vjp.restype = ctypes.c_double
    return L


def p(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(D)


def fd_check(f, x, a, vjp, h=1e-6, rtol=2e-6, atol=1e-11):
    """vjp: J^T a computed by the code under test; f: forward (vector)."""
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros_like(x)
    for k in range(x.size):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        g[k] = np.dot((f(xp) - f(xm)) / (2 * h), a)
    np.testing.assert_allclose(vjp, g, rtol=rtol, atol=atol)


def test_roma_derivatives(lib):
    rng = np.random.default_rng(1)
    r = rng.uniform(-1.6, 1.6, 400)
    r = r[(np.abs(np.abs(r) - 0.5) > 1e-3) & (np.abs(np.abs(r) - 1.5) > 1e-3)]
    h = 1e-6
    for x in r:
        d = (lib.t_phi(x + h) - lib.t_phi(x - h)) / (2 * h)
        assert abs(lib.t_dphi(x) - d) < 1e-7
        dd = (lib.t_dphi(x + h) - lib.t_dphi(x - h)) / (2 * h)
        assert abs(lib.t_ddphi(x) - dd) < 2e-5 * max(1.0, abs(dd))
    # closed forms: phi'' = -1 at 0, 4 just inside 3/2, 0 outside
    assert abs(lib.t_ddphi(0.0) + 1.0) < 1e-15
    assert abs(lib.t_ddphi(1.5 - 1e-12) - 4.0) < 1e-6
    assert lib.t_ddphi(1.6) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_collide_vjp(lib, seed):
    rng = np.random.default_rng(seed)
    tau = rng.uniform(0.55, 1.8)
    omega, pre = 1.0 / tau, 1.0 - 0.5 / tau
    h = 0.02 * rng.standard_normal(9)
    F = 1e-3 * rng.standard_normal(2)
    a = rng.standard_normal(9)
    uh = rng.standard_normal(2)

    def f(z):
        out = np.zeros(11)
        lib.t_collide_fwd(p(z[:9]), z[9], z[10], ctypes.c_double(omega), ctypes.c_double(pre), p(out))
        return out

    out = np.zeros(11)
    lib.t_collide_vjp(p(h), F[0], F[1], ctypes.c_double(omega), ctypes.c_double(pre), p(a),
                      uh[0], uh[1], p(out))
    fd_check(f, np.concatenate([h, F]), np.concatenate([a, uh]), out, h=1e-6)


def test_star_vjp(lib):
    rng = np.random.default_rng(3)
    h = 0.02 * rng.standard_normal(9)
    g = 1e-4 * rng.standard_normal(2)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1.0])
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1.0])

    def f(z):
        rho = 1 + z.sum()
        return np.array([rho, (z @ ex + 0.5 * g[0]) / rho, (z @ ey + 0.5 * g[1]) / rho])

    a = rng.standard_normal(3)
    m = f(h)
    out = np.zeros(9)
    lib.t_star_vjp(ctypes.c_double(m[0]), ctypes.c_double(m[1]), ctypes.c_double(m[2]),
                   ctypes.c_double(a[0]), ctypes.c_double(a[1]), ctypes.c_double(a[2]), p(out))
    fd_check(f, h, a, out)


@pytest.mark.parametrize("seed", range(5))
def test_strain_vjp(lib, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.2, 1.2, 2)
    l0 = rng.uniform(0.5, 1.5)
    ks = rng.uniform(1e-3, 0.1)

    def f(z):
        s = np.zeros(2)
        lib.t_strain_fwd(z[0], z[1], ctypes.c_double(l0), ctypes.c_double(z[2]), p(s))
        return s

    a = rng.standard_normal(2)
    out = np.zeros(3)
    lib.t_strain_vjp(d[0], d[1], ctypes.c_double(l0), ctypes.c_double(ks), a[0], a[1], p(out))
    fd_check(f, np.array([d[0], d[1], ks]), a, out)


@pytest.mark.parametrize("seed", range(8))
def test_bend_vjp(lib, seed):
    rng = np.random.default_rng(seed)
    dL = rng.uniform(0.4, 1.2) * np.array([np.cos(a := rng.uniform(0, 6.28)), np.sin(a)])
    turn = rng.uniform(-1.0, 1.0)
    ang = a + turn
    dR = rng.uniform(0.4, 1.2) * np.array([np.cos(ang), np.sin(ang)])
    th0 = rng.uniform(-0.5, 0.5)
    kb = rng.uniform(1e-3, 1e-1)

    def f(z):
        F = np.zeros(6)
        lib.t_bend_fwd(p(z[:4]), ctypes.c_double(th0), ctypes.c_double(z[4]), p(F))
        return F

    Fh = rng.standard_normal(6)
    out = np.zeros(5)
    x = np.concatenate([dL, dR, [kb]])
    lib.t_bend_vjp(p(x[:4]), ctypes.c_double(th0), ctypes.c_double(kb), p(Fh), p(out))
    fd_check(f, x, Fh, out, rtol=1e-5)


def test_area_vjp(lib):
    rng = np.random.default_rng(9)
    for _ in range(5):
        d = rng.standard_normal(2)
        kap = rng.standard_normal()
        a = rng.standard_normal(2)

        def f(z):
            return z[2] * np.array([z[1], -z[0]])

        out = np.zeros(3)
        lib.t_area_vjp(d[0], d[1], ctypes.c_double(kap), a[0], a[1], p(out))
        fd_check(f, np.array([d[0], d[1], kap]), a, out)


@pytest.mark.parametrize("seed", range(5))
def test_spring_vjp(lib, seed):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1, 1, 2)
    c = np.array([rng.uniform(0, 10), rng.uniform(-0.4, 1.0)])
    r = np.array([rng.uniform(0, 10), -0.5])
    sigma, y_eq = rng.uniform(1e-3, 1e-2), 0.25

    def f(z):
        dd, cc, sg = z[:2], z[2:4], z[4]
        y = np.linalg.norm(cc - r)
        n = np.array([dd[1], -dd[0]]) / np.linalg.norm(dd)
        return sg * (y - y_eq) * n

    a = rng.standard_normal(2)
    y = np.linalg.norm(c - r)
    dy = (c - r) / y
    out = np.zeros(5)
    lib.t_spring_vjp(d[0], d[1], ctypes.c_double(y), ctypes.c_double(dy[0]), ctypes.c_double(dy[1]),
                     ctypes.c_double(sigma), ctypes.c_double(y_eq), a[0], a[1], p(out))
    fd_check(f, np.concatenate([d, c, [sigma]]), a, out)


@pytest.mark.parametrize("seed", range(5))
def test_hydro_vjp(lib, seed):
    rng = np.random.default_rng(seed)
    pr = 1e-3 * rng.standard_normal()
    g = 1e-3 * rng.standard_normal(4)
    nu = 1.0 / 6.0
    ang = rng.uniform(0, 6.28)
    n = np.array([np.cos(ang), np.sin(ang)])
    ln = rng.uniform(0.5, 1.5)

    def f(z):
        F = np.zeros(2)
        lib.t_hydro_fwd(ctypes.c_double(z[0]), p(z[1:5]), ctypes.c_double(nu), ctypes.c_double(z[5]),
                        ctypes.c_double(z[6]), ctypes.c_double(z[7]), p(F))
        return F

    a = rng.standard_normal(2)
    out = np.zeros(8)
    lib.t_hydro_vjp(ctypes.c_double(pr), p(g), ctypes.c_double(nu), ctypes.c_double(n[0]),
                    ctypes.c_double(n[1]), ctypes.c_double(ln), a[0], a[1], p(out))
    fd_check(f, np.concatenate([[pr], g, n, [ln]]), a, out, h=1e-7, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_spring_fwd(lib, seed):
    """Eq. adhFor: sigma (y - y_eq) along the element's outward normal (d_y, -d_x)/|d|."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1, 1, 2)
    y, sigma, y_eq = rng.uniform(0.1, 1.0), rng.uniform(1e-3, 1e-2), 0.25
    F = np.zeros(2)
    lib.t_spring_fwd(d[0], d[1], y, sigma, y_eq, p(F))
    n = np.array([d[1], -d[0]]) / np.hypot(*d)
    np.testing.assert_allclose(F, sigma * (y - y_eq) * n, rtol=1e-14, atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_rigid_load_vjp(lib, seed):
    """Summed load and torque of a rigid particle, F = f, M = r x f."""
    rng = np.random.default_rng(seed)
    r, f = rng.standard_normal(2), rng.standard_normal(2)

    def fwd(z):
        rr, ff = z[:2], z[2:]
        return np.array([ff[0], ff[1], rr[0] * ff[1] - rr[1] * ff[0]])

    a = rng.standard_normal(3)
    out = np.zeros(4)
    lib.t_rigid_load_vjp(r[0], r[1], f[0], f[1], a[0], a[1], a[2], p(out))
    # out = (f^, r^); the forward's inputs are ordered (r, f)
    fd_check(fwd, np.concatenate([r, f]), a, np.concatenate([out[2:], out[:2]]))


@pytest.mark.parametrize("first", [0, 1])
def test_bdf2_vjp(lib, first):
    """Eqs. linearVelRig / angularVelRig: v' = 2/3 (2 v - v_prev/2 + r/m); v + r/m first."""
    m = 3.7

    def fwd(z):
        v, vp, r = z
        return np.array([v + r / m if first else (2.0 / 3.0) * (2.0 * v - 0.5 * vp + r / m)])

    a = np.array([1.3])
    out = np.zeros(2)
    rh = lib.t_bdf2_vjp(first, m, a[0], p(out))
    fd_check(fwd, np.array([0.2, -0.1, 0.05]), a, np.array([out[0], out[1], rh]))


@pytest.mark.parametrize("seed", range(4))
def test_rigid_vertex_vjp(lib, seed):
    """X' = x_c' + R(theta') r0, U_k = U' + Omega' x (X' - x_c')."""
    rng = np.random.default_rng(seed)
    r0 = rng.standard_normal(2) * 3.0
    s = np.array([rng.uniform(0, 50), rng.uniform(0, 20), rng.uniform(-3, 3),
                  1e-2 * rng.standard_normal(), 1e-2 * rng.standard_normal(), 1e-2 * rng.standard_normal()])

    def fwd(z):
        c, sn = np.cos(z[2]), np.sin(z[2])
        rel = np.array([c * r0[0] - sn * r0[1], sn * r0[0] + c * r0[1]])
        X = z[:2] + rel
        U = z[3:5] + z[5] * np.array([-rel[1], rel[0]])
        return np.concatenate([X, U])

    got = np.zeros(4)
    lib.t_rigid_vertex_fwd(r0[0], r0[1], p(s), p(got))
    np.testing.assert_allclose(got, fwd(s), rtol=1e-13, atol=1e-13)
    a = rng.standard_normal(4)
    c, sn = np.cos(s[2]), np.sin(s[2])
    rel = np.array([c * r0[0] - sn * r0[1], sn * r0[0] + c * r0[1]])
    out = np.zeros(6)
    lib.t_rigid_vertex_vjp(rel[0], rel[1], s[5], p(a[:2]), p(a[2:]), p(out))
    fd_check(fwd, s, a, out)
