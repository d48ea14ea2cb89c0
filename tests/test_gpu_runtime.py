"""Runtime features on the GPU: replayed step graphs, the autotuner, state digests and
batch invariance.  Every configuration must give the same bits (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import DELIVERY_ARRIVAL, DELIVERY_PUSH, Simulation
from paper_1511_09325_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _same_as_oracle(sim, p, T, net=0):
    ref = oracle.Sim(p)
    ref.step(T)
    got = sim.read_spikes(net, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(net), ref.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("graph_steps,record", [(16, 100), (16, 40), (7, 100)],
                         ids=["g16-rec-all", "g16-rec-part", "g7"])
def test_graph_steps_bit_exact(graph_steps, record):
    p = W.tiny(3, 4, npc=40, seed=31)
    T = 100
    sim = Simulation(p, record_steps=record, raster_capacity=T * 480)
    sim.set_launch(graph_steps=graph_steps)
    sim.step(T)
    ref = oracle.Sim(p)
    ref.step(T)
    got = sim.read_spikes(0, 0, min(record, T))
    for u in range(min(record, T)):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(0), ref.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("graph_steps", [0, 10])
def test_set_params_reaches_the_next_steps(graph_steps):
    """tau_m and g_AHP changed between steps reach every later step, also when the steps run
    from a captured graph (the constants are kernel arguments by value, so the graph must be
    captured again): the run equals the oracle stepped with the old parameters and then,
    from the same state, with the new ones."""
    p = W.tiny(2, 3, npc=40, seed=33)
    q = dict(p, tau_m=14.0, g_ahp=0.6)
    T1, T2 = 30, 40
    sim = Simulation(p, record_steps=T1 + T2)
    sim.set_launch(graph_steps=graph_steps)
    sim.step(T1)
    sim.set_params(q["tau_m"], q["g_ahp"])
    sim.step(T2)
    a = oracle.Sim(p)
    a.step(T1)
    st = a.state()
    b = oracle.Sim(q)
    b.set_state(T1, st["v"], st["ca"], st["ref"], st["pend"])
    b.step(T2)
    got = sim.read_spikes(0, 0, T1 + T2)
    for u in range(T1):
        assert np.array_equal(got[u], a.spikes(u)), u
    for u in range(T1, T1 + T2):
        assert np.array_equal(got[u], b.spikes(u)), u
    x, y = sim.state(0), b.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(x[k], y[k]), k


def test_graph_after_restore_and_relaunch():
    p = W.tiny(2, 3, npc=40, seed=32)
    sim = Simulation(p, record_steps=90)
    sim.set_launch(graph_steps=10)
    sim.step(30)
    sim.save(1)
    sim.step(20)
    sim.restore(1)
    sim.set_launch(tile=(2, 2), graph_steps=12)
    sim.step(60)
    _same_as_oracle(sim, p, 90)


def test_digest_identical_across_launches():
    p = W.tiny(4, 4, npc=48, seed=33)
    digests = []
    for launch in [dict(delivery=DELIVERY_ARRIVAL, block=1024, tile=(4, 4)),
                   dict(delivery=DELIVERY_ARRIVAL, block=64, tile=(1, 1)),
                   dict(delivery=DELIVERY_ARRIVAL, block=256, tile=(3, 2)),
                   dict(delivery=DELIVERY_PUSH, block=256)]:
        sim = Simulation(p, **launch)
        sim.step(120)
        digests.append(sim.digest())
    assert len(set(digests)) == 1
    other = Simulation(dict(p, seed=34))
    other.step(120)
    assert other.digest() != digests[0]


def test_autotune_keeps_the_trajectory(tmp_path):
    p = W.tiny(4, 5, npc=40, seed=35)
    sim = Simulation(p, record_steps=90)
    sim.step(30)
    cache = str(tmp_path / "tune.jsonl")
    best = sim.autotune(window=10, cache_path=cache)
    assert best["ms_per_step"] > 0
    assert sim.now == 30
    assert sim.get_launch()["block"] == best["block"]
    sim.step(60)
    _same_as_oracle(sim, p, 90)
    # a second tuner call is served from the cache
    sim2 = Simulation(p)
    sim2.step(5)
    best2 = sim2.autotune(window=10, cache_path=cache)
    assert (best2["delivery"], best2["block"], best2["tile"]) == \
        (best["delivery"], best["block"], best["tile"])


def test_batched_members_match_solo_runs_with_graphs():
    nets = W.batched_networks(8, base_seed=40)
    nets = [dict(q, npc=40, n_exc=32) for q in nets]
    T = 120
    batch = Simulation(nets, record_steps=T, raster_capacity=T * 20000)
    batch.set_launch(graph_steps=20)
    batch.step(T)
    for n, p in enumerate(nets):
        solo = Simulation(p, record_steps=T, raster_capacity=T * 5000)
        solo.step(T)
        a, b = batch.read_spikes(n, 0, T), solo.read_spikes(0, 0, T)
        for u in range(T):
            assert np.array_equal(a[u], b[u]), (n, u)
        sa, sb = batch.state(n), solo.state(0)
        for k in ("v", "ca", "ref", "pend"):
            assert np.array_equal(sa[k], sb[k]), (n, k)
        assert batch.stats(n)["e_rec"] == solo.stats(0)["e_rec"]
    for n in (0, 7):
        ref = oracle.Sim(nets[n])
        ref.step(T)
        got = batch.read_spikes(n, 0, T)
        for u in range(T):
            assert np.array_equal(got[u], ref.spikes(u)), (n, u)


@pytest.mark.parametrize("nets", [1, 2], ids=["one-network", "two-networks"])
def test_read_spikes_through_the_abi(nets):
    """sim_read_spikes: a size query (no buffer) answers ETRUNC with the count, a short
    buffer receives its first ids and ETRUNC, and a window in the middle of the record gives
    per-step offsets from zero and the oracle's ids."""
    import ctypes as C
    from paper_1511_09325_amd import _lib as L
    ps = [W.tiny(2, 3, npc=40, seed=51), W.tiny(2, 2, npc=40, seed=52)][:nets]
    T, t0, t1 = 60, 17, 49
    sim = Simulation(ps if nets > 1 else ps[0], record_steps=T)
    sim.step(T)
    ref = oracle.Sim(ps[-1])
    ref.step(T)
    want = np.concatenate([ref.spikes(u) for u in range(t0, t1)]).astype(np.int32)
    off = np.zeros(t1 - t0 + 1, np.int64)
    n = C.c_int64(-1)
    P64, P32 = C.POINTER(C.c_int64), C.POINTER(C.c_int32)
    rc = sim.lib.sim_read_spikes(sim.h, nets - 1, t0, t1, off.ctypes.data_as(P64), None, 0,
                                 C.byref(n))
    assert rc == L.ETRUNC and n.value == len(want) > 10
    short = np.full(10, -7, np.int32)
    rc = sim.lib.sim_read_spikes(sim.h, nets - 1, t0, t1, off.ctypes.data_as(P64),
                                 short.ctypes.data_as(P32), short.size, C.byref(n))
    assert rc == L.ETRUNC and n.value == len(want)
    assert np.array_equal(short, want[:10])
    ids = np.full(len(want), -7, np.int32)
    rc = sim.lib.sim_read_spikes(sim.h, nets - 1, t0, t1, off.ctypes.data_as(P64),
                                 ids.ctypes.data_as(P32), ids.size, C.byref(n))
    assert rc == L.OK and np.array_equal(ids, want)
    assert off[0] == 0 and off[-1] == len(want)
    for u in range(t0, t1):
        assert np.array_equal(ids[off[u - t0]:off[u - t0 + 1]], ref.spikes(u)), u


def test_tune_tiling_picks_an_admissible_shape_that_stays_bit_exact():
    """sim_tune_tiling builds the network once per admissible native tiling; the shapes must
    agree bit for bit (the call checks their digests), and the one it returns runs the
    oracle's raster."""
    from paper_1511_09325_amd import sim as S
    p = W.tiny(4, 5, npc=36, seed=21)
    (tx, ty), ms = S.tune_tiling(p, settle=20, window=30)
    assert (tx, ty) in {(3, 3), (3, 2), (2, 3), (2, 2), (2, 1), (1, 2), (1, 1)} and ms > 0
    T = 80
    sim = Simulation(p, record_steps=T, tile=(tx, ty))
    assert sim.get_launch()["tile"] == (tx, ty)
    sim.step(T)
    ref = oracle.Sim(p)
    ref.step(T)
    got = sim.read_spikes(0, 0, T)
    assert all(np.array_equal(got[u], ref.spikes(u)) for u in range(T))
