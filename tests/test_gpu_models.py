"""The neuron-model variants on the GPU against the oracle, bit for bit: LIF with a second
(sodium-dependent) AHP variable and Izhikevich RS/FS neurons, in both delivery forms, several
tile shapes, several networks in one launch, graph replay and save/restore (needs an MI355X)."""
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


NA = dict(g_na=0.15, tau_na=90.0, na_inc=0.03)
IZH = dict(neuron_model=oracle.NEURON_IZHIKEVICH, j_ext=1.6)


def _same(sim, p, T, net=0):
    ref = oracle.Sim(p)
    ref.step(T)
    got = sim.read_spikes(net, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(net), ref.state()
    for k in ("v", "ca", "ref", "pend", "na"):
        if k == "na" and p.get("g_na", 0.0) == 0.0:
            continue  # the library keeps no sodium variable when it cannot act
        assert np.array_equal(a[k], b[k]), k
    st, rc = sim.stats(net), ref.counts()
    assert (st["spikes"], st["e_rec"], st["e_ext"]) == (rc["spikes"], rc["e_rec"], rc["e_ext"])
    return rc["spikes"]


@pytest.mark.parametrize("model", ["na", "izh"])
@pytest.mark.parametrize("delivery,tile", [(DELIVERY_ARRIVAL, (0, 0)), (DELIVERY_ARRIVAL, (2, 3)),
                                           (DELIVERY_PUSH, (0, 0))],
                         ids=["arrival", "arrival-2x3", "push"])
def test_model_variant_bit_exact(model, delivery, tile):
    extra = NA if model == "na" else IZH
    p = W.tiny(3, 4, npc=48, seed=21, ext_rate_hz=3.4, **extra)
    T = 150
    sim = Simulation(p, record_steps=T, delivery=delivery, tile=tile)
    sim.step(T)
    assert _same(sim, p, T) > 0


@pytest.mark.parametrize("model", ["na", "izh"])
def test_model_variant_batched_graph_and_restore(model):
    extra = NA if model == "na" else IZH
    nets = [W.tiny(2, 2, npc=40, seed=s, ext_rate_hz=r, **extra)
            for s, r in ((3, 3.2), (4, 3.6), (5, 3.4))]
    T = 120
    sim = Simulation(nets, record_steps=T)
    sim.set_launch(graph_steps=10)
    sim.step(40)
    sim.save(2)
    sim.step(30)
    sim.restore(2)
    sim.step(T - 40)
    for n, p in enumerate(nets):
        _same(sim, p, T, net=n)
