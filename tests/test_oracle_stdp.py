"""Pins of the oracle's spike-timing-dependent plasticity (CPU only).

The paper lists STDP among the simulator's features (sections 1-2) and switches it off for
its measurements; it prints no rule.  The reading is the all-to-all pair rule with
exponential windows on the synapses of excitatory sources: every pair of a spike arrival at
the target (emission + delay) and a postsynaptic spike changes the weight once, by
+A+ exp(-(t_post - t_arr) / tau+) when the postsynaptic spike is not earlier than the
arrival, and by -A- exp(-(t_arr - t_post) / tau-) when it is; the weight stays in
[0, w_max]; inhibitory weights stay fixed.  Weights are int16 codes of 2^-14 mV and every
change is rounded to a code where it is applied.  Pinned by:
  * one pair of spikes, swept over the timing difference: the change equals the window's
    closed form (up to one code for the float32 traces);
  * all-to-all: several presynaptic (or postsynaptic) spikes add their window values before
    rounding;
  * the bounds are met exactly and a depressed weight of 0 can grow again; inhibitory
    weights never change;
  * a spike delivers the weight it finds at arrival, so a later arrival carries the changes
    made in between;
  * with A+ = A- = 0 a network runs bit for bit like the same network without plasticity
    (the arrival-form delivery against the push form);
  * on a small network the final weights equal a brute-force replay of the rule from the
    raster: pair sums over the spike times in float64, rounded and clamped event by event.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import workloads as W

Q = 16384.0  # weight codes per mV


def _pair_params(**kw):
    p = W.tiny(1, 1, npc=2, p_own=0.0, p_remote=0.0, ext_rate_hz=0.0, n_exc=2, stdp=1,
               stdp_a_plus=0.05, stdp_a_minus=0.06, stdp_tau_plus=20.0, stdp_tau_minus=30.0,
               stdp_w_max=0.4)
    p.update(kw)
    return p


def _two_neurons(p, d, w_code, pre=0, post=1):
    row_ptr = np.zeros(3, np.int64)
    row_ptr[pre + 1:] = 1
    net = (row_ptr, np.array([post], np.int32), np.array([d], np.uint8),
           np.array([w_code], np.int16))
    sim = oracle.Sim(p, net)
    z = np.zeros(2, np.float32)
    sim.set_state(0, z, z, np.zeros(2, np.uint8), np.zeros((sim.D, 2), np.int32), na=z)
    return sim


def _drive(sim, schedule, steps, record=False):
    """Force the spikes in schedule (neuron -> steps) by 100 mV inputs; returns the spike
    steps of each neuron and, with record, the input each neuron consumed per step."""
    got = {0: [], 1: []}
    if record:
        sim.record(True)
    for u in range(steps):
        for j, ts in schedule.items():
            if u in ts:
                sim.inject(0, j, 100 * 65536)
        sim.step(1)
        for j in sim.spikes(u).tolist():
            got[j].append(u)
    inputs = sim.trajectory(steps)["input"] if record else None
    return got, inputs


def _f32_power(p, k):
    x = np.float32(1.0)
    for _ in range(k):
        x = np.float32(np.float32(p) * x)
    return float(x)


@pytest.mark.parametrize("dt", list(range(-40, 41, 3)) + [0, -1, 1])
def test_single_pair_window(dt):
    p = _pair_params()
    d, w0 = 4, 1638
    t_pre = 50
    t_arr = t_pre + d
    t_post = t_arr + dt
    sim = _two_neurons(p, d, w0)
    got, _ = _drive(sim, {0: [t_pre], 1: [t_post]}, 160)
    assert got == {0: [t_pre], 1: [t_post]}
    w = int(sim.weights()[0])
    if dt >= 0:
        exact = p["stdp_a_plus"] * math.exp(-dt / p["stdp_tau_plus"]) * Q
        f32 = p["stdp_a_plus"] * _f32_power(math.exp(-1 / p["stdp_tau_plus"]), dt) * Q
        want = w0 + round(exact)
    else:
        exact = p["stdp_a_minus"] * math.exp(dt / p["stdp_tau_minus"]) * Q
        f32 = p["stdp_a_minus"] * _f32_power(math.exp(-1 / p["stdp_tau_minus"]), -dt) * Q
        want = w0 - round(exact)
    assert abs(w - want) <= 1, (dt, w, want)
    assert abs(f32 - exact) < 0.01 * max(exact, 1)
    # the size of the change falls off with |dt| at the window's rate
    if abs(dt) >= 3:
        assert abs(abs(w - w0) - exact) <= 0.5 + 1e-6


def test_all_to_all_sums_before_rounding():
    p = _pair_params()
    d, w0 = 3, 2000
    pp = math.exp(-1 / 20.0)
    pm = math.exp(-1 / 30.0)
    # two arrivals, then one postsynaptic spike: one change of A+ (P^a + P^b)
    sim = _two_neurons(p, d, w0)
    got, _ = _drive(sim, {0: [10, 17], 1: [31]}, 80)
    assert got == {0: [10, 17], 1: [31]}
    want = w0 + round(0.05 * Q * (pp ** (31 - 13) + pp ** (31 - 20)))
    assert abs(int(sim.weights()[0]) - want) <= 1
    # two postsynaptic spikes, then one arrival: one change of -A- (P^a + P^b)
    sim = _two_neurons(p, d, w0)
    got, _ = _drive(sim, {0: [30], 1: [10, 20]}, 80)
    assert got == {0: [30], 1: [10, 20]}
    want = w0 - round(0.06 * Q * (pm ** (33 - 10) + pm ** (33 - 20)))
    assert abs(int(sim.weights()[0]) - want) <= 1
    # one arrival, two postsynaptic spikes after it: two changes, each rounded
    sim = _two_neurons(p, d, w0)
    _drive(sim, {0: [10], 1: [15, 25]}, 80)
    want = w0 + round(0.05 * Q * pp ** 2) + round(0.05 * Q * pp ** 12)
    assert abs(int(sim.weights()[0]) - want) <= 2


def test_bounds_and_regrowth():
    p = _pair_params(stdp_w_max=0.2)
    qmax = round(0.2 * Q)
    sim = _two_neurons(p, 2, qmax - 100)
    _drive(sim, {0: [10], 1: [12]}, 40)          # +819 codes, clamped
    assert int(sim.weights()[0]) == qmax
    sim = _two_neurons(p, 2, 300)
    # post at 21 then arrival at 22: -951 codes -> 0; the post spike at 62 meets the
    # arrivals at 62 and (all-to-all) at 22
    _drive(sim, {0: [20, 60], 1: [21, 62]}, 100)
    w = int(sim.weights()[0])
    assert abs(w - round(0.05 * Q * (1.0 + math.exp(-40 / 20.0)))) <= 1
    sim = _two_neurons(p, 2, 300)
    _drive(sim, {0: [20], 1: [21]}, 40)
    assert int(sim.weights()[0]) == 0


def test_inhibitory_weights_do_not_change():
    p = _pair_params(n_exc=1)            # neuron 1 inhibitory, weight negative
    sim = _two_neurons(p, 2, -3000, pre=1, post=0)
    got, _ = _drive(sim, {1: [10, 30], 0: [13, 25, 40]}, 80)
    assert got == {0: [13, 25, 40], 1: [10, 30]}
    assert int(sim.weights()[0]) == -3000


def test_a_spike_delivers_the_weight_it_finds():
    p = _pair_params()
    d, w0 = 5, 1000
    sim = _two_neurons(p, d, w0)
    got, inputs = _drive(sim, {0: [10, 30], 1: [20]}, 60, record=True)
    assert got == {0: [10, 30], 1: [20]}
    assert inputs[15, 1] == 4 * w0
    w1 = w0 + round(0.05 * Q * math.exp(-5 / 20.0))    # post at 20, arrival at 15
    assert abs(inputs[35, 1] // 4 - w1) <= 1
    w2 = inputs[35, 1] // 4 - round(0.06 * Q * math.exp(-15 / 30.0))  # post 20, arrival 35
    assert abs(int(sim.weights()[0]) - w2) <= 1
    assert inputs[36:, 1].sum() == 0 and inputs[:15, 1].sum() == 0


@pytest.mark.parametrize("seed", [1, 2])
def test_zero_amplitudes_equal_the_static_network(seed):
    base = W.tiny(2, 2, npc=30, seed=seed, ext_rate_hz=3.4)
    a = oracle.Sim(dict(base))
    b = oracle.Sim(dict(base, stdp=1, stdp_a_plus=0.0, stdp_a_minus=0.0))
    T = 250
    a.step(T)
    b.step(T)
    assert a.counts()["spikes"] > 0
    assert all(np.array_equal(x, y) for x, y in zip(a.raster(0, T), b.raster(0, T)))
    sa, sb = a.state(), b.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(sa[k], sb[k]), k
    assert a.counts() == b.counts() and a.consumed() == b.consumed()
    assert np.array_equal(a.weights(), b.weights())


def _replay(p, net, raster, T):
    """The rule replayed from the spike times: every arrival meets the postsynaptic spikes
    before it (depression), every postsynaptic spike the arrivals up to it (potentiation);
    pair sums in float64; at one step depression comes before potentiation."""
    row_ptr, tgt, dly, wq = net
    n = len(row_ptr) - 1
    posts = [[] for _ in range(n)]
    pres = [[] for _ in range(n)]
    for u in range(T):
        for j in raster[u].tolist():
            posts[j].append(u)
            pres[j].append(u)
    a_p, a_m = p["stdp_a_plus"] * Q, p["stdp_a_minus"] * Q
    t_p, t_m = p["stdp_tau_plus"], p["stdp_tau_minus"]
    qmax = round(p["stdp_w_max"] * Q)
    out = wq.astype(np.int64).copy()
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            w = int(wq[e])
            if w < 0 or not pres[i]:
                continue
            j, d = int(tgt[e]), int(dly[e])
            arr = [t + d for t in pres[i] if t + d < T]
            events = sorted([(t, 0) for t in arr] + [(t, 1) for t in posts[j]])
            for t, kind in events:
                if kind == 0:
                    dw = round(a_m * sum(math.exp(-(t - s) / t_m) for s in posts[j] if s < t))
                    w = max(0, w - dw)
                else:
                    dw = round(a_p * sum(math.exp(-(t - s) / t_p) for s in arr if s <= t))
                    w = min(qmax, w + dw)
            out[e] = w
    return out


@pytest.mark.parametrize("seed", [3, 4])
def test_weights_equal_a_replay_from_the_raster(seed):
    p = W.tiny(2, 2, npc=24, seed=seed, ext_rate_hz=3.4, stdp=1, stdp_a_plus=0.02,
               stdp_a_minus=0.021)
    net = oracle.network(p)
    sim = oracle.Sim(p, net)
    T = 300
    sim.step(T)
    raster = sim.raster(0, T)
    assert sim.counts()["spikes"] > 50
    got = sim.weights().astype(np.int64)
    want = _replay(p, net, raster, T)
    diff = np.abs(got - want)
    changed = got != net[3]
    assert changed.sum() > 100                   # the rule did act
    assert np.all(got[net[3] < 0] == net[3][net[3] < 0])
    assert diff.max() <= 3 and (diff == 0).mean() > 0.99, (diff.max(), (diff == 0).mean())


def test_single_synapse_replay_equals_the_simulation():
    """oracle.stdp_synapse, which the full-size GPU checks use one synapse at a time, gives
    every synapse of a simulated network its final weight bit for bit."""
    p = W.tiny(2, 2, npc=24, seed=6, ext_rate_hz=3.4, stdp=1, stdp_a_plus=0.03,
               stdp_a_minus=0.032, stdp_w_max=0.25)
    net = oracle.network(p)
    sim = oracle.Sim(p, net)
    T = 260
    sim.step(T)
    n = oracle.n_neurons(p)
    spk = np.zeros((n, T), np.uint8)
    for u, ids in enumerate(sim.raster(0, T)):
        spk[ids, u] = 1
    row_ptr, tgt, dly, wq = net
    got = sim.weights()
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            want = oracle.stdp_synapse(p, spk[i], spk[tgt[e]], int(dly[e]), int(wq[e]))
            assert got[e] == want, (i, e)
    assert (got != wq).sum() > 100 and (got == round(0.25 * Q)).any()
