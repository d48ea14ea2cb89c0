"""Parity at the full 24x24 and 96x96 grids (needs an MI355X).

The 24x24 grid's first 200 steps are compared with the whole oracle (its network of 885M
synapses is built on every host thread, about 20-40 s).  Beyond that, and at 96x96 (14.2G
synapses), each check uses only what the oracle can compute one by one, in the launch
configuration that bench.py times (arrival form, default workgroup and tile), early in the
run and late in it, where the network fires at its steady rate (tens of Hz, bursty) and the
gather windows, work-ordered tiles and large per-tile spike counts are all in play:
  * synapse rows of sampled source neurons, bit for bit against the generator's definition;
  * the pending input of sampled target neurons at sampled steps, bit for bit against the
    brute-force sum over every candidate synapse whose source spiked (from the GPU raster);
  * one whole step of all N neurons: the oracle updates every neuron from the GPU's state
    and pending input, and V, Ca, the refractory counters and the spike list after the
    GPU's step must be identical.
"""
import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import Simulation
from paper_1511_09325_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _sample_rows(p, n, rng, k):
    npc = p["npc"]
    ncol = p["rows"] * p["cols"]
    fixed = [0, n - 1, npc - 1, npc, p["n_exc"] - 1, p["n_exc"], (ncol - 1) * npc,
             (p["cols"] - 1) * npc + 5, (ncol // 2) * npc + npc // 2]
    return sorted(set(fixed) | set(rng.choice(n, size=k, replace=False).tolist()))


def _check_rows(sim, p, rows):
    for i in rows:
        rp, tgt, dly, wq = sim.synapses(0, i, i + 1)
        otgt, odly, owq = oracle.row(p, i)
        assert np.array_equal(tgt, otgt), i
        assert np.array_equal(dly, odly), i
        assert np.array_equal(wq, owq), i


def _spot_step(sim, p, u, rng, n_targets):
    """Advance to step u, check sampled pending inputs against brute force, then check the
    whole step u of every neuron against the oracle's update."""
    n = oracle.n_neurons(p)
    dmax = p["d_max"]
    sim.step(u - sim.now)
    st = sim.state()
    # spikes of the steps whose synapses can still be pending: [u - dmax, u)
    t0 = max(0, u - dmax)
    mask = np.zeros((u - t0, n), np.uint8)
    for e, ids in enumerate(sim.read_spikes(0, t0, u)):
        mask[e, ids] = 1
    targets = np.array(_sample_rows(p, n, rng, n_targets), np.int64)
    for q in (0, 1, dmax - 1):
        want = oracle.input_brute(p, targets, u + q, u - 1, mask, t0)
        got = st["pend"][q][targets]
        assert np.array_equal(got, want), (u, q, np.flatnonzero(got != want)[:5])
    spk, v, ca, ref = oracle.update_many(p, u, st["pend"][0], st["v"], st["ca"], st["ref"])
    del st, mask
    sim.step(1)
    after = sim.state(pend=False)
    assert np.array_equal(sim.read_spikes(0, u, u + 1)[0], np.flatnonzero(spk))
    assert np.array_equal(after["ref"], ref)
    assert np.array_equal(after["v"], v), np.abs(after["v"] - v).max()
    assert np.array_equal(after["ca"], ca), np.abs(after["ca"] - ca).max()
    return int(spk.sum())


LATE_24 = (1000, 1001)   # a gathering step of the window and the light step after it
LATE_96 = (1500, 1501)


@pytest.fixture(scope="module")
def sim24():
    p = W.PLAIN_24X24["params"]
    sim = Simulation(p, record_steps=LATE_24[-1] + 1)
    yield p, sim
    sim.close()


def test_24x24_rows(sim24):
    p, sim = sim24
    _check_rows(sim, p, _sample_rows(p, sim.n_neurons, np.random.default_rng(24), 60))


@pytest.mark.parametrize("u", [3, 40, 150])
def test_24x24_spot_steps(sim24, u):
    p, sim = sim24
    spikes = _spot_step(sim, p, u, np.random.default_rng(u), 800)
    if u >= 40:
        assert spikes > 0


def test_24x24_first_200_steps_equal_the_oracle(sim24):
    """The whole 24x24 network in the oracle: the GPU raster of steps 0-199 and the state
    after step 199 (V, Ca, refractory counters, pending input) equal it bit for bit."""
    import oracle as O
    p, sim = sim24
    T = 200
    assert sim.now <= T
    sim.step(T - sim.now)
    ref = O.Sim(p)
    ref.step(T)
    got = sim.read_spikes(0, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(0), ref.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(a[k], b[k]), k
    st, rc = sim.stats(0), ref.counts()
    assert (st["spikes"], st["e_rec"], st["e_ext"]) == (rc["spikes"], rc["e_rec"], rc["e_ext"])
    assert rc["spikes"] > 0


@pytest.mark.parametrize("u", LATE_24)
def test_24x24_late_spot_steps(sim24, u):
    p, sim = sim24
    launch = sim.get_launch()
    assert launch["gather_steps"] > 1 and LATE_24[0] % launch["gather_steps"] == 0
    spikes = _spot_step(sim, p, u, np.random.default_rng(u), 800)
    assert spikes > 0.002 * sim.n_neurons  # the steady state: some Hz at least


@pytest.fixture(scope="module")
def sim96():
    p = W.PLAIN_96X96["params"]
    sim = Simulation(p, record_steps=LATE_96[-1] + 1)
    yield p, sim
    sim.close()
    import torch
    torch.cuda.empty_cache()


def test_96x96_rows(sim96):
    p, sim = sim96
    _check_rows(sim, p, _sample_rows(p, sim.n_neurons, np.random.default_rng(96), 40))


@pytest.mark.parametrize("u", [30, 70])
def test_96x96_spot_steps(sim96, u):
    p, sim = sim96
    spikes = _spot_step(sim, p, u, np.random.default_rng(u), 300)
    assert spikes > 0


@pytest.mark.parametrize("u", LATE_96)
def test_96x96_late_spot_steps(sim96, u):
    """Step 1500 (a gathering step of the three-step window) and step 1501 (the light step
    after it), three quarters into the 2 s run: the regime bench.py times."""
    p, sim = sim96
    launch = sim.get_launch()
    assert launch["gather_steps"] > 1 and LATE_96[0] % launch["gather_steps"] == 0
    spikes = _spot_step(sim, p, u, np.random.default_rng(u), 300)
    assert spikes > 0.005 * sim.n_neurons  # the steady state fires at tens of Hz


def test_batched_workload_members_equal_their_plain_runs():
    """The batched workload itself (64 networks of the full column recipe, grids 2x2..8x8,
    external rates 2-6 Hz, 2.5G synapses), stepped with the bench's launch (one launch per
    step, graph chunks of 50): after 100 steps every member's raster, V, Ca, refractory
    counters, pending input and counters equal those of the same network run alone."""
    nets = W.batched_networks(64, 0)
    T = 100
    batch = Simulation(nets, record_steps=T)
    batch.set_launch(graph_steps=50)
    batch.step(T)
    batch.sync()
    for n, p in enumerate(nets):
        solo = Simulation(p, record_steps=T)
        solo.step(T)
        a, b = batch.read_spikes(n, 0, T), solo.read_spikes(0, 0, T)
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), n
        sa, sb = batch.state(n), solo.state(0)
        for k in ("v", "ca", "ref", "pend"):
            assert np.array_equal(sa[k], sb[k]), (n, k)
        ca, cb = batch.stats(n), solo.stats(0)
        assert (ca["spikes"], ca["e_rec"], ca["e_ext"]) == (cb["spikes"], cb["e_rec"], cb["e_ext"]), n
        solo.close()
    batch.close()
