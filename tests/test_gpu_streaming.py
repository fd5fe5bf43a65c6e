"""The two population streaming forms on the GPU: two buffers (pull from one,
write the other) and one buffer updated in place (a pass that reads and
writes each node's neighbours alternating with a pass local to the node).

The collision and the pulled values are the same in both, so every result
must be the same bit for bit: fields, markers, bonds, the state blob, the
adjoint's gradient; and converting a running context from one form to the
other must not change its trajectory."""
import numpy as np
import pytest

import paper_1907_00080_amd as pkg
from paper_1907_00080_amd.adjoint import AdjointWindow
from workloads import configs

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-streaming] {msg}", flush=True)


def _cases():
    out = []
    adh = configs.small_case(nx=64, ny=24, n_rbc=0, adhesive=True, seed_offset=31,
                             particles=(configs.PARTICLE_SOFT, configs.PARTICLE_RIGID))
    out.append(("adhesive", adh))
    zh = configs.small_case(nx=72, ny=30, n_rbc=1, particles=(configs.PARTICLE_RIGID,),
                            seed_offset=32)
    zh.walls = "zou-he"
    zh.u_wall = (0.0, 0.01)
    out.append(("zou-he walls", zh))
    out.append(("periodic", configs.small_case(nx=72, ny=40, n_rbc=1, periodic_y=1,
                                               particles=(configs.PARTICLE_SOFT,), seed_offset=33)))
    mls = configs.small_case(nx=96, ny=24, n_rbc=1, particles=(configs.PARTICLE_RIGID,),
                             seed_offset=34)
    mls.transfer = "mls"
    out.append(("mls", mls))
    rep = configs.small_case(nx=129, ny=33, n_rbc=2, particles=(configs.PARTICLE_RIGID,),
                             seed_offset=35)
    rep.repulsion = configs.REPULSION_COEFF
    out.append(("repulsion", rep))
    return out


def _same(a, b, wl):
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
    for k in range(len(wl.bodies)):
        assert np.array_equal(a.markers(k), b.markers(k)), k
    assert np.array_equal(a.bonds(), b.bonds())


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_in_place_equals_two_buffers_on_small_cases(dtype):
    for name, wl in _cases():
        announce(f"{name} {dtype}")
        runs = []
        for mode in (0, 1):
            s = pkg.Sim(wl, dtype=dtype, graph_steps=6, streaming=mode)
            assert s.streaming == mode
            s.step(25)
            d = s.diagnostics()
            assert d["nonfinite"] == 0 and d["bin_overflow"] == 0
            runs.append(s)
        _same(runs[0], runs[1], wl)
        for s in runs:
            s.close()


def test_in_place_equals_two_buffers_capillary_and_batch():
    wl = configs.capillary_2000x200()
    announce("capillary 2000x200, tile 32x8, 41 steps")
    a = pkg.Sim(wl, dtype="f32", tile=(32, 8), graph_steps=10, streaming=0)
    b = pkg.Sim(wl, dtype="f32", tile=(32, 8), graph_steps=10, streaming=1)
    a.step(41)
    b.step(41)
    _same(a, b, wl)
    a.close()
    b.close()
    ws = [w for _, w in _cases()[:3]]
    for i, w in enumerate(ws):
        w.instance = i
    announce("uneven batch")
    ba = pkg.Batch(ws, dtype="f32", graph_steps=10, streaming=0)
    bb = pkg.Batch(ws, dtype="f32", graph_steps=10, streaming=1)
    assert ba.streaming == 0 and bb.streaming == 1
    ba.step(33)
    bb.step(33)
    for i, w in enumerate(ws):
        for x, y in zip(ba.fields(i), bb.fields(i)):
            assert np.array_equal(x, y), i
        for k in range(len(w.bodies)):
            assert np.array_equal(ba.markers(i, k), bb.markers(i, k)), (i, k)
    ba.close()
    bb.close()


def test_state_blob_and_conversion_between_forms():
    """A blob saved by one form restores into the other at either parity; a
    running context converted between forms keeps its trajectory; the
    lattice-kernel timing call leaves an in-place state unchanged."""
    wl = _cases()[0][1]
    announce("state blob and conversion")
    ref = pkg.Sim(wl, dtype="f64", graph_steps=0, streaming=0)
    ref.step(7)
    blob = ref.get_state()
    ref.step(12)
    for restore_at in (0, 1):       # parity of the context that restores
        s = pkg.Sim(wl, dtype="f64", graph_steps=0, streaming=1)
        s.step(restore_at + 2)
        s.set_state(blob)
        s.step(12)
        _same(ref, s, wl)
        assert s.get_state() == ref.get_state()
        s.close()
    s = pkg.Sim(wl, dtype="f64", graph_steps=4, streaming=1)
    s.step(5)
    s.set_streaming(0)
    assert s.streaming == 0
    s.step(4)
    s.set_streaming(1)
    s.step(3)
    s.time_lattice_kernel(3)
    s.step(7)
    _same(ref, s, wl)
    ref.close()
    s.close()


def test_adjoint_gradient_same_in_both_forms():
    wl = configs.adjoint_channel(nx=96, ny=32, seed_offset=6)
    announce("adjoint window in both forms")
    grads = []
    for mode in (0, 1):
        sim = pkg.Sim(wl, dtype="f64", streaming=mode)
        sim.step(1)
        win = AdjointWindow(sim, 20, 6)
        J, _ = win.forward()
        grads.append((J, win.backward(1.0)))
        sim.close()
    assert grads[0][0] == grads[1][0]
    assert np.array_equal(grads[0][1], grads[1][1])
