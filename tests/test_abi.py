"""C-ABI checks that need no GPU: the library loads, exports every entry point
the headers declare, and rejects bad arguments and wrong-phase calls before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1907_00080_amd as pkg
from workloads import configs, geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("lbib.h", "lbib_batch.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(lbib_[a-z_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = pkg.library()
    decl = _declared()
    assert len(decl) >= 30
    for name in decl:
        assert hasattr(lib, name), name
    assert decl == set(pkg.EXPORTS)
    header = open(os.path.join(ROOT, "include", "lbib.h")).read()
    want = int(re.search(r"#define LBIB_ABI_VERSION (\d+)u", header).group(1))
    assert lib.lbib_abi_version() == want
    for s, n in pkg.STATUS.items():
        assert lib.lbib_status_string(s).decode() == n


def _desc(**kw):
    d = dict(nx=16, ny=8, periodic_y=0, dtype=0, tau=1.0, gx=0.0, gy=0.0, seed=1, instance=0,
             tile_x=0, tile_y=0)
    d.update(kw)
    return pkg.LatticeDesc(**d)


def _create(**kw):
    lib = pkg.library()
    h = ctypes.c_void_p()
    st = lib.lbib_create(ctypes.byref(_desc(**kw)), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw", [dict(nx=0), dict(ny=0), dict(tau=0.5), dict(tau=float("nan")),
                                dict(dtype=7), dict(tile_x=48, tile_y=4)])
def test_create_rejects_bad_lattice(kw):
    st, h = _create(**kw)
    assert st == 1 and not h.value
    assert pkg.library().lbib_last_error(None)


def test_body_and_receptor_validation_and_phases():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    try:
        ccw = geometry.place(geometry.circle(2.0, 12), 0.0, [8.0, 4.0])
        bd = pkg.BodyDesc(2, 12, 0.0, 0.0, 1.0, 1 / 3, 1.1, 0.0, 0)
        bid = ctypes.c_int32()
        ok = np.ascontiguousarray(ccw)
        assert lib.lbib_add_body(h, ctypes.byref(bd), ok.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.byref(bid)) == 0 and bid.value == 0
        cw = np.ascontiguousarray(ccw[::-1])
        assert lib.lbib_add_body(h, ctypes.byref(bd), cw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 None) == 1
        bd.nv = 2
        assert lib.lbib_add_body(h, ctypes.byref(bd), ok.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 None) == 1
        bad = np.array([0.0, 3.0, 2.0])
        assert lib.lbib_set_receptors(h, 0, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3) == 1
        good = np.array([0.0, 2.0, 3.5])
        assert lib.lbib_set_receptors(h, 0, good.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3) == 0
        assert lib.lbib_set_receptors(h, 2, good.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 3) == 1
        out = np.array([0.0, 16.0])
        assert lib.lbib_set_receptors(h, 1, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2) == 1
        # running-phase calls refused during set-up (no device work happens)
        assert lib.lbib_step(h, 1) == 2
        assert lib.lbib_get_fields(h, None, None, None) == 2
        assert lib.lbib_finalize_setup(h) == 2
        nb = ctypes.c_size_t()
        assert lib.lbib_workspace_query(h, ctypes.byref(nb)) == 0 and nb.value > 16 * 8 * 9 * 4
        # misaligned and undersized workspaces are refused before any device use
        assert lib.lbib_bind(h, ctypes.c_void_p(4096 + 8), nb.value, None) == 1
        assert lib.lbib_bind(h, ctypes.c_void_p(4096), nb.value - 1, None) == 4
        assert lib.lbib_set_graph_steps(h, 3) == 1
        assert lib.lbib_set_graph_steps(h, 4) == 0
        assert lib.lbib_last_error(h)
    finally:
        assert lib.lbib_destroy(h) == 0
    assert lib.lbib_destroy(None) == 0


def test_workspace_grows_with_lattice_and_dtype():
    lib = pkg.library()
    sizes = {}
    for dt in (0, 1):
        for nx in (64, 640):
            st, h = _create(nx=nx, ny=32, dtype=dt)
            nb = ctypes.c_size_t()
            assert lib.lbib_workspace_query(h, ctypes.byref(nb)) == 0
            sizes[(dt, nx)] = nb.value
            lib.lbib_destroy(h)
    # populations A, B (9 each) and velocity (2): 20 values per node
    assert sizes[(0, 640)] - sizes[(0, 64)] >= 20 * 4 * 576 * 32
    assert sizes[(1, 640)] - sizes[(1, 64)] >= 20 * 8 * 576 * 32


def test_batch_create_rules():
    lib = pkg.library()
    a, ha = _create()
    b, hb = _create(dtype=1)
    arr = (ctypes.c_void_p * 2)(ha.value, hb.value)
    out = ctypes.c_void_p()
    assert lib.lbib_batch_create(arr, 2, 0, 0, ctypes.byref(out)) == 1   # dtype mismatch
    c, hc = _create(nx=40)
    arr = (ctypes.c_void_p * 2)(ha.value, hc.value)
    assert lib.lbib_batch_create(arr, 2, 0, 0, ctypes.byref(out)) == 0
    n = ctypes.c_int32()
    assert lib.lbib_batch_size(out, ctypes.byref(n)) == 0 and n.value == 2
    bd = pkg.BodyDesc(0, 12, 0.0, 0.0, 1.0, 1 / 3, 1.0, 0.0, 0)
    xy = np.ascontiguousarray(geometry.place(geometry.circle(2.0, 12), 0.0, [8.0, 4.0]))
    assert lib.lbib_add_body(out, ctypes.byref(bd), xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             None) == 2
    for h in (ha, hb, hc, out):
        lib.lbib_destroy(h)


def test_product_path_requires_built_library(monkeypatch):
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", "/nonexistent/liblbib.so")
    with pytest.raises(ImportError):
        pkg.Sim(configs.small_case(nx=16, ny=8, n_rbc=0))


def test_adjoint_calls_need_a_running_single_context():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    n = ctypes.c_size_t()
    assert lib.lbib_adjoint_workspace_query(h, 10, 5, ctypes.byref(n)) == 2
    assert lib.lbib_adjoint_workspace_query(h, 0, 5, ctypes.byref(n)) == 1
    assert lib.lbib_adjoint_workspace_query(h, 10, 0, ctypes.byref(n)) == 1
    assert lib.lbib_adjoint_bind(h, None, 0, 10, 5) == 1
    J = ctypes.c_double()
    assert lib.lbib_adjoint_forward(h, ctypes.byref(J), None) == 2
    g = (ctypes.c_double * 3)()
    assert lib.lbib_adjoint_backward(h, 1.0, g) == 2
    assert lib.lbib_set_body_params(h, 0, 1.0, 0.0, 0.0) == 2
    lib.lbib_destroy(h)


def test_step_mode_validation():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    assert lib.lbib_set_step_mode(h, 4) == 1
    assert lib.lbib_set_step_mode(h, -1) == 1
    for m in (0, 1, 2, 3):
        assert lib.lbib_set_step_mode(h, m) == 0
        got = ctypes.c_int32()
        assert lib.lbib_get_step_mode(h, ctypes.byref(got)) == 0
        assert got.value == m
    lib.lbib_destroy(h)


def test_lattice_launch_validation():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    got = ctypes.c_int32()
    assert lib.lbib_get_lattice_launch(h, ctypes.byref(got)) == 0 and got.value == 0
    for bad in (-1, 3, 5, 16):
        assert lib.lbib_set_lattice_launch(h, bad) == 1
    for w in (1, 2, 4, 8, 0):
        assert lib.lbib_set_lattice_launch(h, w) == 0
        assert lib.lbib_get_lattice_launch(h, ctypes.byref(got)) == 0 and got.value == w
    assert lib.lbib_get_lattice_launch(h, None) == 1
    lib.lbib_destroy(h)


def test_streaming_validation():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    got = ctypes.c_int32()
    for bad in (-2, 2, 7):
        assert lib.lbib_set_streaming(h, bad) == 1
    for mode, want in ((0, 0), (1, 1)):
        assert lib.lbib_set_streaming(h, mode) == 0
        assert lib.lbib_get_streaming(h, ctypes.byref(got)) == 0 and got.value == want
    # automatic: a small lattice's one population buffer fits the last-level cache
    assert lib.lbib_set_streaming(h, -1) == 0
    assert lib.lbib_get_streaming(h, ctypes.byref(got)) == 0 and got.value == 1
    assert lib.lbib_get_streaming(h, None) == 1
    lib.lbib_destroy(h)


def test_repulsion_validation_and_phase():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    try:
        assert lib.lbib_set_repulsion(h, -1e-6, 2.0) == 1
        assert lib.lbib_set_repulsion(h, float("nan"), 2.0) == 1
        assert lib.lbib_set_repulsion(h, 1e-5, 0.0) == 1
        assert lib.lbib_set_repulsion(h, 1e-5, 17.0) == 1
        assert lib.lbib_set_repulsion(h, 1e-5, float("inf")) == 1
        assert lib.lbib_set_repulsion(h, configs.REPULSION_COEFF, 2.0) == 0
        assert lib.lbib_set_repulsion(h, 0.0, 2.0) == 0      # off
        assert lib.lbib_set_repulsion(None, 1e-5, 2.0) == 1
    finally:
        lib.lbib_destroy(h)


def test_observation_calls_need_a_running_context():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    assert lib.lbib_observe(h) == 2
    assert lib.lbib_reset_observations(h) == 2
    rec = (pkg.BodyObs * 1)()
    assert lib.lbib_get_observations(h, rec) == 2
    assert lib.lbib_get_observations(h, None) == 1
    assert lib.lbib_observe(None) == 1
    lib.lbib_destroy(h)


def test_wall_mode_validation():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    try:
        assert lib.lbib_set_walls(h, 2, 0.0, 0.0) == 1
        assert lib.lbib_set_walls(h, 0, 0.0, 0.01) == 1          # moving walls need mode 1
        assert lib.lbib_set_walls(h, 1, 0.0, 0.5) == 1           # |u| > 0.3
        assert lib.lbib_set_walls(h, 1, float("nan"), 0.0) == 1
        assert lib.lbib_set_walls(h, 1, 0.0, 0.01) == 0
        assert lib.lbib_set_walls(h, 0, 0.0, 0.0) == 0
    finally:
        lib.lbib_destroy(h)
    st, h = _create(periodic_y=1)
    assert lib.lbib_set_walls(h, 1, 0.0, 0.0) == 1               # no walls to move
    lib.lbib_destroy(h)
    st, h = _create(ny=1)
    assert lib.lbib_set_walls(h, 1, 0.0, 0.0) == 1
    lib.lbib_destroy(h)


def test_transfer_validation():
    lib = pkg.library()
    st, h = _create()
    assert st == 0
    try:
        assert lib.lbib_set_transfer(h, 2, 1, 1.3) == 1                 # unknown mode
        assert lib.lbib_set_transfer(h, 1, 3, 1.3) == 1                 # unknown weight
        assert lib.lbib_set_transfer(h, 1, 1, 1.0) == 1                 # support must exceed 1
        assert lib.lbib_set_transfer(h, 1, 2, 1.51) == 1                # and lie within 3/2
        assert lib.lbib_set_transfer(h, 1, 1, float("nan")) == 1
        assert lib.lbib_set_transfer(h, 1, 0, float("nan")) == 0        # ignored for the Roma weight
        assert lib.lbib_set_transfer(h, 1, 1, 1.3) == 0
        assert lib.lbib_set_transfer(h, 1, 2, 1.5) == 0
        assert lib.lbib_set_transfer(h, 0, 1, 1.3) == 0
        assert lib.lbib_set_transfer(None, 0, 1, 1.3) == 1
    finally:
        lib.lbib_destroy(h)


def test_workload_transfer_is_checked_before_any_device_work():
    from workloads import configs as c
    wl = c.Workload("t", 16, 8)
    wl.transfer = "spline"
    with pytest.raises(ValueError):
        pkg.Sim(wl, dtype="f64", device="cpu")
