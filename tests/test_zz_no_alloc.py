"""sim_read_spikes_static (the allocation-free variant of sim_read_spikes) against
sim_read_spikes, through the C ABI: identical offsets, ids, counts and return codes, on two
calls in a row of which the second reads a smaller range, for several networks in one
simulation (the path that uses the scratch array) and for a single network."""
import ctypes as C

import numpy as np
import pytest

from paper_1511_09325_amd import _lib as L
from paper_1511_09325_amd import Simulation
from paper_1511_09325_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _read(fn, sim, net, t0, t1, cap):
    off = np.full(t1 - t0 + 1, -7, np.int64)
    ids = np.full(max(cap, 1), -7, np.int32)
    n = C.c_int64(-1)
    rc = fn(sim.h, net, t0, t1, off.ctypes.data_as(C.POINTER(C.c_int64)),
            ids.ctypes.data_as(C.POINTER(C.c_int32)), cap, C.byref(n))
    return rc, off, ids[:min(cap, max(n.value, 0))], n.value


def _same(sim, net, t0, t1, cap=None):
    lib = L.lib()
    if cap is None:
        cap = _read(lib.sim_read_spikes, sim, net, t0, t1, 0)[3]
    a = _read(lib.sim_read_spikes, sim, net, t0, t1, cap)
    b = _read(lib.sim_read_spikes_static, sim, net, t0, t1, cap)
    assert a[0] == b[0], (a[0], b[0])
    assert a[3] == b[3]
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    return a


def test_static_read_matches_allocating_read_several_networks():
    nets = [W.tiny(2, 2, npc=48, seed=3), W.tiny(3, 2, npc=48, seed=4),
            W.tiny(2, 3, npc=48, seed=5)]
    T = 120
    sim = Simulation(nets, record_steps=T)
    sim.step(T)
    sim.sync()
    first = _same(sim, 1, 0, T)
    assert first[0] == L.OK and first[3] > 0
    # a second, smaller call: another network over a shorter window
    second = _same(sim, 2, 10, 40)
    assert second[0] == L.OK and 0 < second[3] < first[3]
    # a short ids buffer: ETRUNC with the same count and the same first ids
    short = _same(sim, 0, 0, T, cap=5)
    assert short[0] == L.ETRUNC
    # an empty range
    assert _same(sim, 0, 7, 7)[3] == 0


def test_static_read_matches_allocating_read_one_network():
    p = W.tiny(3, 3, npc=40, seed=8)
    T = 90
    sim = Simulation(p, record_steps=T)
    sim.step(T)
    sim.sync()
    a = _same(sim, 0, 0, T)
    b = _same(sim, 0, 30, 50)
    assert a[0] == b[0] == L.OK and 0 < b[3] < a[3]
