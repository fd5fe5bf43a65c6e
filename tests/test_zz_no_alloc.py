"""Allocation-free field readback (lbib_get_fields_noalloc) against
lbib_get_fields, called through the C ABI: two calls in a row, the second on a
smaller lattice, then the first lattice again; and the staging limit."""
import ctypes

import numpy as np
import pytest

import paper_1907_00080_amd as pkg
from workloads import configs

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


def _noalloc(sim):
    n = sim.nx * sim.ny
    out = [np.full(n, np.nan) for _ in range(3)]
    p = [o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for o in out]
    st = sim.lib.lbib_get_fields_noalloc(sim.h, p[0], p[1], p[2])
    return st, [o.reshape(sim.ny, sim.nx) for o in out]


def _same(sim):
    st, got = _noalloc(sim)
    assert st == 0, sim.lib.lbib_last_error(sim.h).decode()
    for a, b in zip(got, sim.fields()):
        assert np.array_equal(a, b)


def test_noalloc_fields_match_get_fields():
    big = configs.small_case(nx=200, ny=40, n_rbc=2,
                             particles=(configs.PARTICLE_RIGID, configs.PARTICLE_SOFT))
    announce(f"{big.name} f32, then a smaller f64 lattice, then the first again")
    a = pkg.Sim(big, dtype="f32")
    a.step(30)
    _same(a)
    small = configs.small_case(nx=64, ny=24, n_rbc=1, particles=(configs.PARTICLE_SOFT,))
    b = pkg.Sim(small, dtype="f64")
    b.step(10)
    _same(b)
    a.step(5)
    _same(a)


def test_noalloc_rejects_lattice_beyond_staging():
    wl = configs.Workload("beyond-staging", 1024, 520, periodic_y=1)   # 532480 > 2^19 nodes
    announce(f"{wl.name} {wl.nx}x{wl.ny}")
    sim = pkg.Sim(wl, dtype="f32")
    st, _ = _noalloc(sim)
    assert st == 1
    assert "staging" in sim.lib.lbib_last_error(sim.h).decode()
