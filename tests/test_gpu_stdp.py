"""Spike-timing-dependent plasticity on the GPU against the oracle (needs an MI355X).

The tile kernel depresses each plastic record as it delivers it and writes the traces; a
second kernel potentiates the synapses into the step's spiking neurons through the reverse
index.  Checked:
  * small networks (both connectivity kernels, several tilings, all three neuron models):
    raster, state, counters and every weight bit for bit against the oracle;
  * two networks in one launch under graph replay and a change of workgroup size;
  * A+ = A- = 0: the same raster and state as the network without plasticity;
  * snapshots hold the weights and traces (save, run, restore, run again: same digest);
  * launch changes that would break the rule's one-owner write-back are refused;
  * the full 24x24 grid: whole steps of every neuron against the oracle's update from the
    GPU state, and the final weights of every synapse of sampled rows against the rule
    replayed one synapse at a time from the GPU raster.
"""
import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import Simulation
from paper_1511_09325_amd import workloads as W

pytestmark = pytest.mark.gpu

STRONG = dict(stdp=1, stdp_a_plus=0.02, stdp_a_minus=0.021, stdp_w_max=0.3)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _same(sim, p, T, net=0, check_weights=True):
    ref = oracle.Sim(p)
    ref.step(T)
    got = sim.read_spikes(net, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(net), ref.state()
    for k in ("v", "ca", "ref", "pend") + (("na",) if p["g_na"] != 0 else ()):
        assert np.array_equal(a[k], b[k]), k
    st, rc = sim.stats(net), ref.counts()
    assert (st["spikes"], st["e_rec"], st["e_ext"]) == (rc["spikes"], rc["e_rec"], rc["e_ext"])
    if check_weights:
        rp, tgt, dly, wq = sim.synapses(net)
        orp, otgt, odly, owq = oracle.network(p)
        assert np.array_equal(rp, orp) and np.array_equal(tgt, otgt)
        w = ref.weights()
        bad = np.flatnonzero(wq != w)
        assert bad.size == 0, (bad[:5], wq[bad[:5]], w[bad[:5]])
        assert (w != owq).sum() > 0.05 * len(w)  # the rule did act
    return rc["spikes"]


CASES = {
    "2x2": (W.tiny(2, 2, npc=40, seed=1, **STRONG), (0, 0)),
    "4x4-tile2x2": (W.tiny(4, 4, npc=36, seed=2, **STRONG), (2, 2)),
    "3x5-tile1x1": (W.tiny(3, 5, npc=30, seed=3, **STRONG), (1, 1)),
    "paper-7x8": (dict(W.paper_grid(7, 8, 4, npc=36, n_exc=29), ext_rate_hz=3400.0 / 540.0,
                       wi_mu=-0.8, wi_sigma=0.08, **STRONG), (0, 0)),
    "sodium-3x3": (W.tiny(3, 3, npc=32, seed=5, g_na=0.1, tau_na=100.0, na_inc=0.02,
                          **STRONG), (0, 0)),
    "izhikevich-2x3": (W.tiny(2, 3, npc=30, seed=6, j_ext=1.6,
                              neuron_model=oracle.NEURON_IZHIKEVICH, **STRONG), (0, 0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_stdp_bit_exact(name):
    p, tile = CASES[name]
    T = 160
    sim = Simulation(p, record_steps=T, tile=tile)
    assert sim.get_launch()["gather_steps"] == 1
    sim.step(T)
    assert _same(sim, p, T) > 0


def test_stdp_batched_graph_and_block_change():
    nets = [W.tiny(3, 3, npc=30, seed=7, **STRONG), W.tiny(2, 4, npc=30, seed=8, **STRONG)]
    T = 120
    sim = Simulation(nets, record_steps=T)
    sim.set_launch(graph_steps=10)
    sim.step(40)
    sim.set_launch(block=256)
    sim.step(40)
    sim.set_launch(block=512, graph_steps=0)
    sim.step(T - 80)
    for n, p in enumerate(nets):
        _same(sim, p, T, net=n)


def test_zero_amplitudes_equal_the_static_network():
    base = W.tiny(3, 4, npc=40, seed=9)
    T = 150
    a = Simulation(base, record_steps=T)
    b = Simulation(dict(base, stdp=1, stdp_a_plus=0.0, stdp_a_minus=0.0), record_steps=T)
    a.step(T)
    b.step(T)
    assert all(np.array_equal(x, y) for x, y in zip(a.read_spikes(), b.read_spikes()))
    sa, sb = a.state(), b.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.synapses(0)[3], b.synapses(0)[3])
    assert a.stats()["spikes"] > 0


def test_snapshot_holds_weights_and_traces():
    p = W.tiny(3, 3, npc=36, seed=10, **STRONG)
    sim = Simulation(p, record_steps=200)
    sim.step(50)
    sim.save(3)
    d50 = sim.digest()
    sim.step(60)
    d110, w110 = sim.digest(), sim.synapses(0)[3].copy()
    sim.restore(3)
    assert sim.digest() == d50
    sim.step(60)
    assert sim.digest() == d110
    assert np.array_equal(sim.synapses(0)[3], w110)
    assert not np.array_equal(w110, oracle.network(p)[3])


def test_launch_changes_that_break_the_rule_are_refused():
    from paper_1511_09325_amd import DELIVERY_PUSH
    p = W.tiny(4, 4, npc=30, seed=11, **STRONG)
    sim = Simulation(p)
    other = (2, 2) if sim.get_launch()["tile"] != (2, 2) else (1, 1)
    for kw in (dict(delivery=DELIVERY_PUSH), dict(tile=other), dict(gather_steps=2)):
        with pytest.raises(RuntimeError, match="STDP"):
            sim.set_launch(**kw)
    sim.set_launch(block=128)
    sim.step(5)
    with pytest.raises(RuntimeError, match="STDP"):
        Simulation(p, gather_steps=3)


# ---- full 24x24 grid ----------------------------------------------------------------------
T24 = 301


@pytest.fixture(scope="module")
def stdp24():
    p = dict(W.PLAIN_24X24["params"], stdp=1)
    sim = Simulation(p, record_steps=T24 + 1)
    yield p, sim
    sim.close()


def _whole_step(sim, p, u):
    """Step u of every neuron against the oracle's update from the GPU's state and pending
    input (with plasticity the pending input is what the emitted spikes bring with today's
    weights; the input of step u is consumed before any of them changes)."""
    sim.step(u - sim.now)
    st = sim.state()
    spk, v, ca, ref = oracle.update_many(p, u, st["pend"][0], st["v"], st["ca"], st["ref"])
    del st
    sim.step(1)
    after = sim.state(pend=False)
    assert np.array_equal(sim.read_spikes(0, u, u + 1)[0], np.flatnonzero(spk))
    assert np.array_equal(after["ref"], ref)
    assert np.array_equal(after["v"], v)
    assert np.array_equal(after["ca"], ca)
    return int(spk.sum())


@pytest.mark.parametrize("u", [40, 250])
def test_24x24_whole_steps(stdp24, u):
    p, sim = stdp24
    assert _whole_step(sim, p, u) > 0


def test_24x24_weights_of_sampled_rows_equal_the_rule(stdp24):
    p, sim = stdp24
    sim.step(T24 - sim.now)
    n = sim.n_neurons
    spk = np.zeros((n, T24), np.uint8)
    for u, ids in enumerate(sim.read_spikes(0, 0, T24)):
        spk[ids, u] = 1
    rng = np.random.default_rng(24)
    npc = p["npc"]
    rows = sorted(set(rng.choice(n, size=24, replace=False).tolist()) |
                  {0, npc - 1, p["n_exc"] - 1, n - 1})
    changed = 0
    qmax = round(p["stdp_w_max"] * 16384)
    for i in rows:
        rp, tgt, dly, wq = sim.synapses(0, i, i + 1)
        otgt, odly, owq = oracle.row(p, i)
        assert np.array_equal(tgt, otgt) and np.array_equal(dly, odly)
        for e in range(len(tgt)):
            want = oracle.stdp_synapse(p, spk[i], spk[tgt[e]], int(dly[e]), int(owq[e]))
            assert wq[e] == want, (i, e, int(wq[e]), want)
        changed += int((wq != owq).sum())
        if owq[0] < 0:
            assert np.array_equal(wq, owq)
        else:
            assert wq.min() >= 0 and wq.max() <= max(qmax, owq.max())
    assert changed > 1000
