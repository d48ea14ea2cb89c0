"""GPU path vs the CPU oracle, element by element (needs an MI355X).

Integer results (synapse store, spike rasters, pending input, counters) must be
bit-identical; the float32 state (V, Ca) too, since both sides evaluate the same pinned
float32 expression without contraction (the tolerance ceiling of 1e-5 mV is never needed;
the tests assert equality).
"""
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


def _check_network(sim, p, net=0):
    rp, tgt, dly, wq = sim.synapses(net)
    orp, otgt, odly, owq = oracle.network(p)
    assert np.array_equal(rp, orp)
    assert np.array_equal(tgt, otgt)
    assert np.array_equal(dly, odly)
    assert np.array_equal(wq, owq)


def _check_run(sim, ref, T, net=0, t0=0):
    got = sim.read_spikes(net, t0, T)
    for u in range(t0, T):
        want = ref.spikes(u)
        assert np.array_equal(got[u - t0], want), "raster differs at step %d" % u
    a, b = sim.state(net), ref.state()
    assert np.array_equal(a["ref"], b["ref"])
    assert np.array_equal(a["v"], b["v"]), np.abs(a["v"] - b["v"]).max()
    assert np.array_equal(a["ca"], b["ca"]), np.abs(a["ca"] - b["ca"]).max()
    assert np.array_equal(a["pend"], b["pend"])
    st, rc = sim.stats(net), ref.counts()
    assert (st["spikes"], st["e_rec"], st["e_ext"]) == (rc["spikes"], rc["e_rec"], rc["e_ext"])


@pytest.mark.parametrize("p", [
    W.tiny(2, 5, npc=40, seed=1),
    W.tiny(3, 3, npc=37, seed=2),
    W.tiny(1, 1, npc=50, seed=3),
    W.tiny(4, 4, npc=64, seed=4),
    W.tiny(2, 3, npc=40, seed=5, d_min=3, d_max=7),
], ids=["2x5", "3x3-npc37", "1x1", "4x4", "2x3-d3..7"])
def test_generator_bitwise_tiny(p):
    sim = Simulation(p)
    _check_network(sim, p)


def test_generator_bitwise_2x2_recipe():
    p = W.PLAIN_2X2["params"]
    sim = Simulation(p)
    assert sim.n_synapses == len(oracle.network(p)[1])
    _check_network(sim, p)


@pytest.mark.parametrize("delivery,block,tile", [
    (DELIVERY_ARRIVAL, 64, (1, 1)), (DELIVERY_ARRIVAL, 256, (2, 3)),
    (DELIVERY_ARRIVAL, 1024, (4, 4)), (DELIVERY_ARRIVAL, 128, (3, 1)),
    (DELIVERY_PUSH, 64, (0, 0)), (DELIVERY_PUSH, 1024, (0, 0)),
], ids=["arr-64-1x1", "arr-256-2x3", "arr-1024-4x4", "arr-128-3x1", "push-64", "push-1024"])
def test_tiny_run_bit_exact(delivery, block, tile):
    p = W.tiny(5, 7, npc=40, seed=11)
    T = 300
    sim = Simulation(p, delivery=delivery, block=block, tile=tile, record_steps=T)
    sim.step(T)
    ref = oracle.Sim(p)
    ref.step(T)
    assert ref.counts()["spikes"] > 100
    _check_run(sim, ref, T)


@pytest.mark.parametrize("delivery", [DELIVERY_ARRIVAL, DELIVERY_PUSH], ids=["arrival", "push"])
def test_plain_2x2_one_second_bit_exact(delivery):
    """The 2x2 workload (4,960 neurons, ~6.15M synapses), 1 s at dt = 1 ms."""
    p = W.PLAIN_2X2["params"]
    T = W.PLAIN_2X2["steps"]
    sim = Simulation(p, delivery=delivery, record_steps=T)
    sim.step(T)
    ref = oracle.Sim(p)
    ref.step(T)
    _check_run(sim, ref, T)


def test_batched_members_equal_their_oracle_runs():
    nets = [W.tiny(2, 2, npc=40, seed=0), W.tiny(3, 2, npc=40, seed=1, ext_rate_hz=3.0),
            W.tiny(1, 4, npc=40, seed=2, ext_rate_hz=4.0), W.tiny(3, 3, npc=40, seed=3)]
    T = 200
    sim = Simulation(nets, record_steps=T)
    sim.step(T)
    for n, p in enumerate(nets):
        ref = oracle.Sim(p)
        ref.step(T)
        _check_run(sim, ref, T, net=n)


def test_save_restore_and_switching_delivery():
    p = W.tiny(2, 2, npc=48, seed=21)
    T = 150
    ref = oracle.Sim(p)
    ref.step(T)
    sim = Simulation(p, record_steps=T, delivery=DELIVERY_ARRIVAL, block=128)
    sim.step(50)
    sim.save(3)
    sim.step(30)
    sim.restore(3)            # back to step 50
    assert sim.now == 50
    sim.step(25)
    sim.set_launch(DELIVERY_PUSH, 512)     # ring rebuilt from the spike history
    sim.step(40)
    sim.set_launch(DELIVERY_ARRIVAL, 64, (1, 2))
    sim.step(T - 115)
    got = sim.read_spikes(0, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(0), ref.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("over", [
    dict(p_own=0.0, p_remote=0.0, ext_rate_hz=0.0),      # silent: no synapses, no drive
    dict(d_min=5, d_max=5),                               # a single delay
    dict(t_ref=0),                                        # no refractory period
    dict(ext_rate_hz=20.0),                               # lambda = 20 per step
    dict(npc=1, n_exc=1, rows=1, cols=1),                 # one neuron, no synapse
    dict(n_exc=0),                                        # all inhibitory
    dict(d_min=1, d_max=32),                              # the longest ring
    dict(npc=4096, n_exc=3277, rows=1, cols=1),           # the largest column (12-bit index);
                                                          # on a 1x1 torus every pair connects
], ids=["silent", "one-delay", "tref0", "lambda20", "one-neuron", "all-inh", "dmax32",
        "npc4096"])
@pytest.mark.parametrize("delivery", [DELIVERY_ARRIVAL, DELIVERY_PUSH], ids=["arrival", "push"])
def test_edge_cases(over, delivery):
    p = W.tiny(2, 2, npc=40, seed=7)
    p.update(over)
    T = 120
    n = p["rows"] * p["cols"] * p["npc"]
    sim = Simulation(p, delivery=delivery, record_steps=T, raster_capacity=T * n)
    sim.step(T)
    ref = oracle.Sim(p)
    ref.step(T)
    _check_run(sim, ref, T)


def test_raster_overflow_is_reported():
    p = W.tiny(2, 2, npc=40, seed=1, ext_rate_hz=6.0)
    sim = Simulation(p, record_steps=100, raster_capacity=10)
    sim.step(100)
    from paper_1511_09325_amd import DpsnnError
    with pytest.raises(DpsnnError) as e:
        sim.sync()
    assert e.value.code == -5


def test_plain_4x4_half_second_bit_exact():
    """The forward+backward workload's network (4x4 grid, full column recipe, 24.6M
    synapses), 500 steps, against the oracle; the train-mode forward too."""
    p = W.FWD_BWD_4X4["params"]
    T = W.FWD_BWD_4X4["steps"]
    ref = oracle.Sim(p)
    ref.step(T)
    for train in (False, True):
        sim = Simulation(p, record_steps=T, train_mode=train, ckpt_every=50)
        sim.step(T)
        _check_run(sim, ref, T)
        sim.close()


@pytest.mark.parametrize("native,other", [((2, 2), (3, 3)), ((3, 2), (1, 1)), ((4, 4), (2, 3))],
                         ids=["2x2->3x3", "3x2->1x1", "4x4->2x3"])
def test_tiles_other_than_the_storage_tiling(native, other):
    """The synapse store is split by the tiling chosen at creation; a different tiling
    later reads parts that reach several of its tiles and keeps only its own synapses."""
    p = W.tiny(6, 7, npc=40, seed=17)
    T = 160
    ref = oracle.Sim(p)
    ref.step(T)
    sim = Simulation(p, record_steps=T, tile=native)
    sim.step(60)
    sim.set_launch(tile=other)
    sim.step(T - 60)
    _check_run(sim, ref, T)


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_gather_windows_bit_exact(K):
    """Gathering the input of K steps in one pass over the spike history (adjacent delay
    groups, one accumulator per step) gives the same run for every window."""
    p = W.tiny(5, 7, npc=40, seed=11)
    T = 230
    ref = oracle.Sim(p)
    ref.step(T)
    sim = Simulation(p, record_steps=T, gather_steps=K)
    assert sim.get_launch()["gather_steps"] == K
    sim.step(T)
    _check_run(sim, ref, T)


def test_gather_window_interrupted():
    """Restores, launch changes and graph chunks that start inside a gather window."""
    p = W.tiny(4, 5, npc=40, seed=19)
    T = 200
    ref = oracle.Sim(p)
    ref.step(T)
    sim = Simulation(p, record_steps=T, gather_steps=4)
    sim.step(41)                      # inside the window that starts at step 40
    sim.save(1)
    sim.step(23)
    sim.restore(1)                    # back to step 41
    sim.step(6)
    sim.set_launch(graph_steps=7)     # chunks of 7 steps across windows of 4
    sim.step(70)
    sim.set_launch(gather_steps=3, graph_steps=0)
    sim.step(T - 117)
    _check_run(sim, ref, T)


@pytest.mark.parametrize("rows,cols,graph", [(24, 24, 0), (24, 24, 9), (15, 20, 0)],
                         ids=["576-direct", "576-graph9", "300-direct"])
def test_more_tiles_than_resident_workgroups(rows, cols, graph):
    """Grids of 1x1 tiles in 1024-thread workgroups, one per compute unit, and 512-thread ones
    at the steps inside a window, two per compute unit.  576 tiles are more than the device
    holds workgroups at once for either launch, so every launch hands tiles out from its
    device counter (direct launches and graph chunks that cross gather windows); 300 tiles
    are more only for the gathering launches, whose counter then alternates with light
    launches of one workgroup per tile."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    assert rows * cols > n_cu
    assert (rows * cols > 2 * n_cu) == (rows * cols == 576)
    p = W.tiny(rows, cols, npc=40, seed=23)
    T = 300
    ref = oracle.Sim(p)
    ref.step(T)
    sim = Simulation(p, block=1024, tile=(1, 1), record_steps=T, gather_steps=4)
    if graph:
        sim.set_launch(graph_steps=graph)
    sim.step(T)
    assert ref.counts()["spikes"] > 10000
    _check_run(sim, ref, T)
