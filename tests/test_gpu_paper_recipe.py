"""The paper's own column recipe on the GPU (Gaussian lateral kernel over the 7x7 stencil,
0.8 local pair probability, 540 external synapses; section 2, Methods) against the oracle:
the generated synapses bit for bit, then rasters, states and counters bit for bit on tiny
networks (wrapped and unwrapped stencils, both delivery forms, native and foreign tilings,
several networks per launch), and spot steps of the full 24x24 grid (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import DELIVERY_ARRIVAL, DELIVERY_PUSH, Simulation
from paper_1511_09325_amd import workloads as W

from test_gpu_fullsize import _check_rows, _sample_rows, _spot_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _tiny(rows, cols, npc=32, seed=0, **kw):
    p = W.paper_grid(rows, cols, seed, npc=npc, n_exc=int(round(0.8 * npc)))
    p.update(ext_rate_hz=3400.0 / 540.0, wi_mu=-0.8, wi_sigma=0.08)  # small nets need drive
    p.update(kw)
    return p


@pytest.mark.parametrize("rows,cols", [(2, 2), (3, 5), (8, 9)])
def test_generated_network_equals_the_oracle(rows, cols):
    p = _tiny(rows, cols, npc=24, seed=rows * 10 + cols)
    sim = Simulation(p)
    rp, tgt, dly, wq = sim.synapses(0)
    orp, otgt, odly, owq = oracle.network(p)
    assert np.array_equal(rp, orp)
    assert np.array_equal(tgt, otgt) and np.array_equal(dly, odly) and np.array_equal(wq, owq)
    # once the grid holds the stencil without wrapping, every target column lies inside it
    # (the 7x7 square minus its corners) and the nearest columns are reached
    if rows >= 7 and cols >= 7:
        src = np.repeat(np.arange(len(rp) - 1), np.diff(rp)) // p["npc"]
        tc = tgt // p["npc"]
        dy = (tc // cols - src // cols + rows // 2) % rows - rows // 2
        dx = (tc % cols - src % cols + cols // 2) % cols - cols // 2
        assert np.all((np.abs(dy) <= 3) & (np.abs(dx) <= 3) & (np.abs(dy) + np.abs(dx) < 6))
        assert len(set(zip(dy.tolist(), dx.tolist()))) >= 21


def _same(sim, p, T, net=0):
    ref = oracle.Sim(p)
    ref.step(T)
    got = sim.read_spikes(net, 0, T)
    for u in range(T):
        assert np.array_equal(got[u], ref.spikes(u)), u
    a, b = sim.state(net), ref.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(a[k], b[k]), k
    st, rc = sim.stats(net), ref.counts()
    assert (st["spikes"], st["e_rec"], st["e_ext"]) == (rc["spikes"], rc["e_rec"], rc["e_ext"])
    return rc["spikes"]


@pytest.mark.parametrize("rows,cols,delivery,tile", [
    (4, 4, DELIVERY_ARRIVAL, (0, 0)),
    (7, 8, DELIVERY_ARRIVAL, (0, 0)),
    (7, 8, DELIVERY_ARRIVAL, (2, 2)),
    (7, 8, DELIVERY_PUSH, (0, 0)),
    (9, 6, DELIVERY_ARRIVAL, (3, 2)),
], ids=["4x4", "7x8", "7x8-tile2x2", "7x8-push", "9x6-tile3x2"])
def test_paper_recipe_dynamics_bit_exact(rows, cols, delivery, tile):
    p = _tiny(rows, cols, npc=36, seed=rows + cols)
    T = 120
    sim = Simulation(p, record_steps=T, delivery=delivery, tile=tile)
    sim.step(T)
    assert _same(sim, p, T) > 0


def test_paper_recipe_foreign_tiling_and_batched():
    """Two paper-recipe networks in one launch, switched to a tiling other than the one the
    store was split for (parts then reach several tiles) and back, with graph replay."""
    nets = [_tiny(5, 7, npc=30, seed=3), _tiny(8, 4, npc=30, seed=4)]
    T = 100
    sim = Simulation(nets, record_steps=T)
    sim.set_launch(graph_steps=10)
    sim.step(30)
    sim.set_launch(tile=(1, 1))
    sim.step(40)
    sim.set_launch(tile=(2, 3))
    sim.step(T - 70)
    for n, p in enumerate(nets):
        _same(sim, p, T, net=n)


def test_paper_recipe_more_tiles_than_resident_workgroups():
    """The 7x7 stencil launched over 600 single-column tiles (a 20x30 grid, a tiling other
    than the store's) in 1024-thread workgroups: more tiles than the device holds workgroups
    at once at both launch shapes (one per compute unit gathering, two inside a window), so
    tiles come from the launch's device counter."""
    import torch
    assert 600 > 2 * torch.cuda.get_device_properties(0).multi_processor_count
    p = _tiny(20, 30, npc=24, seed=29)
    T = 150
    sim = Simulation(p, record_steps=T, block=1024)
    sim.set_launch(tile=(1, 1), gather_steps=3)
    assert sim.get_launch()["tile"] == (1, 1) and sim.get_launch()["gather_steps"] == 3
    sim.step(T)
    assert _same(sim, p, T) > 1000


def test_tiling_with_parts_of_more_than_nine_columns_is_refused():
    p = _tiny(8, 8, npc=20)
    with pytest.raises(RuntimeError, match="9 columns"):
        Simulation(p, tile=(4, 4))


@pytest.fixture(scope="module")
def paper24():
    p = W.paper_grid(24, 24, 0)
    sim = Simulation(p, record_steps=302)
    yield p, sim
    sim.close()


def test_paper_24x24_rows(paper24):
    p, sim = paper24
    _check_rows(sim, p, _sample_rows(p, sim.n_neurons, np.random.default_rng(5), 30))
    info_deg = sim.n_synapses / sim.n_neurons
    assert 1235 < info_deg < 1245  # Table 1: 1239-1245 recurrent synapses per neuron


@pytest.mark.parametrize("u", [60, 300, 301])
def test_paper_24x24_spot_steps(paper24, u):
    p, sim = paper24
    spikes = _spot_step(sim, p, u, np.random.default_rng(u), 200)
    if u >= 300:
        assert spikes > 0
