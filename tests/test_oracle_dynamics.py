"""Pins of the oracle's simulation step (CPU only).

The step is the paper's mixed time/event-driven update (section 1): every neuron is
integrated every 1 ms step -- a leaky integrate-and-fire neuron with calcium-driven
after-hyperpolarisation (section 2) -- and each spike reaches its targets through delayed
synapses.  Nothing in the paper prints a trajectory, so the step is pinned here by what
mathematics fixes: closed forms of the leak, of constant drive and of calcium decay, the
refractory interval, the exact arrival of one synapse at every delay, conservation of
delivered input, a brute-force recomputation of every input from the raster, and
invariance to the order of synapses.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import workloads as W

U = 2.0**-16


def _silent(n=8, **kw):
    """No synapses and no external drive unless overridden."""
    p = W.tiny(1, 1, npc=n, p_own=0.0, p_remote=0.0, ext_rate_hz=0.0)
    p.update(kw)
    return p


def _empty_net(n):
    return (np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint8),
            np.zeros(0, np.int16))


def test_initial_potential_range():
    p = W.grid(2, 2, 3)
    v = np.array([oracle.initial_v(p, j) for j in range(2000)])
    assert v.min() >= 0.0 and v.max() < 15.0
    assert abs(v.mean() - 7.5) < 4 * 15 / math.sqrt(12 * 2000)


def test_subthreshold_decay_closed_form():
    """No input and no calcium: V_t = V_0 exp(-t dt / tau_m)."""
    p = _silent()
    sim = oracle.Sim(p, _empty_net(8))
    v0 = sim.state()["v"].astype(np.float64)
    for t in range(1, 201):
        sim.step(1)
        v = sim.state()["v"].astype(np.float64)
        want = v0 * math.exp(-t / 20.0)
        # float32 constant and per-step rounding: at most 2 ulp-relative per step
        assert np.all(np.abs(v - want) <= 2 * t * 2**-24 * want + 1e-30)
    assert sim.counts()["spikes"] == 0


def _drive(sim, j, a, steps):
    """Inject a constant input a (2^-16 mV) into neuron j for `steps` steps; return spike steps."""
    out = []
    for _ in range(steps):
        sim.inject(0, j, a)
        u = sim.now
        sim.step(1)
        if j in set(sim.spikes(u).tolist()):
            out.append(u)
    return out


def _crossing(v_start, i_mv, pm):
    """Smallest m >= 1 with pm^m v_start + i (1 - pm^m)/(1 - pm) >= 20, and the margin."""
    m = 1
    while True:
        v = pm**m * v_start + i_mv * (1 - pm**m) / (1 - pm)
        if v >= 20.0:
            prev = pm ** (m - 1) * v_start + i_mv * (1 - pm ** (m - 1)) / (1 - pm)
            return m, min(v - 20.0, 20.0 - prev)
        m += 1


def test_constant_drive_first_spike_and_isi():
    """Constant drive without AHP: the first spike and every inter-spike interval follow the
    closed form V_m = pm^m V_start + I (1 - pm^m)/(1 - pm); the interval is the refractory
    period (2 steps) plus the climb from V_reset."""
    p = _silent(g_ahp=0.0)
    n = 8
    sim = oracle.Sim(p, _empty_net(n))
    st = sim.state()
    sim.set_state(0, np.zeros(n), np.zeros(n), np.zeros(n), st["pend"] * 0)
    a = 1_500_000                 # about 22.9 mV/step asymptote, 1.5 tau away
    i_mv = a * U
    pm = math.exp(-1 / 20.0)
    spikes = _drive(sim, 3, a, 120)
    m1, margin1 = _crossing(0.0, i_mv, pm)
    k, margin2 = _crossing(15.0, i_mv, pm)
    assert min(margin1, margin2) > 1e-3       # far from any rounding tie
    want = [m1 - 1]
    while want[-1] + 2 + k < 120:
        want.append(want[-1] + 2 + k)
    assert spikes == want
    # a neuron never driven stays silent
    assert all(3 == j for u in range(120) for j in sim.spikes(u))


def test_threshold_is_inclusive():
    p = _silent(g_ahp=0.0)
    sim = oracle.Sim(p, _empty_net(2))
    z = np.zeros(2)
    sim.set_state(0, z, z, z, np.zeros((21, 2), np.int32))
    sim.inject(0, 0, 20 * 65536)          # V = 0 * pm - 0 + 20.0 exactly
    sim.inject(0, 1, 20 * 65536 - 1)      # one unit below
    sim.step(1)
    assert sim.spikes(0).tolist() == [0]


def test_adaptation_lengthens_intervals():
    """With the calcium AHP the interval sequence under constant drive never shortens and
    ends longer than it starts (spike-frequency adaptation, section 2)."""
    p = _silent()
    n = 4
    sim = oracle.Sim(p, _empty_net(n))
    sim.set_state(0, np.zeros(n), np.zeros(n), np.zeros(n), np.zeros((21, n), np.int32))
    spikes = _drive(sim, 1, 85_197, 1500)       # about 1.3 mV per step
    isi = np.diff(spikes)
    assert len(isi) > 20
    assert np.all(np.diff(isi) >= 0)
    assert isi[-1] > isi[0]


def test_calcium_closed_form_and_refractory_discard():
    """Forced spikes at known steps: Ca(u) = sum_k alpha P_c^(u - t_k) after the step.
    A forced input arriving 1 or 2 steps after a spike is discarded (refractory)."""
    p = _silent()
    n = 2
    sim = oracle.Sim(p, _empty_net(n))
    sim.set_state(0, np.zeros(n), np.zeros(n), np.zeros(n), np.zeros((21, n), np.int32))
    forced = [3, 4, 5, 10, 40, 41, 43, 100]       # 4, 5 and 41 fall in refractory periods
    expect_spk = [3, 10, 40, 43, 100]
    big = 100 * 65536
    got = []
    for u in range(300):
        if u in forced:
            sim.inject(0, 0, big)
        sim.step(1)
        if 0 in set(sim.spikes(u).tolist()):
            got.append(u)
        ca = sim.state()["ca"][0]
        want = sum(0.05 * math.exp(-(u - t) / 300.0) for t in expect_spk if t <= u)
        assert abs(ca - want) < 1e-6
    assert got == expect_spk


@pytest.mark.parametrize("d", list(range(1, 21)))
def test_single_synapse_arrives_after_its_delay(d):
    p = _silent()
    wq = -1234
    net = (np.array([0, 1, 1], np.int64), np.array([1], np.int32), np.array([d], np.uint8),
           np.array([wq], np.int16))
    sim = oracle.Sim(p, net)
    z = np.zeros(2)
    sim.set_state(0, z, z, z, np.zeros((21, 2), np.int32))
    sim.record(True)
    u0 = 7
    sim.step(u0)
    sim.inject(0, 0, 100 * 65536)
    sim.step(1)
    assert sim.spikes(u0).tolist() == [0]
    pend = sim.state()["pend"]
    want = np.zeros_like(pend)
    want[d - 1, 1] = 4 * wq
    assert np.array_equal(pend, want)
    sim.step(25)
    inp = sim.trajectory(u0 + 26)["input"][:, 1]
    hot = np.nonzero(inp)[0].tolist()
    assert hot == [u0 + d] and inp[u0 + d] == 4 * wq


@pytest.fixture(scope="module")
def tiny_run():
    p = W.tiny(2, 3, npc=40, seed=4)
    net = oracle.network(p)
    sim = oracle.Sim(p, net)
    sim.record(True)
    T = 300
    sim.step(T)
    return p, net, sim, T


def test_tiny_network_is_active(tiny_run):
    p, net, sim, T = tiny_run
    c = sim.counts()
    rate = c["spikes"] / (oracle.n_neurons(p) * T * 1e-3)
    assert 1.0 < rate < 200.0


def test_brute_force_input_and_counts(tiny_run):
    """Every consumed input equals the sum over all synapses whose source spiked exactly
    one delay earlier, plus the external count times J_ext; the counters equal the raster."""
    p, (row_ptr, tgt, dly, wq), sim, T = tiny_run
    n = oracle.n_neurons(p)
    s = np.zeros((T, n), np.int64)
    for u in range(T):
        s[u, sim.spikes(u)] = 1
    traj = sim.trajectory(T)
    assert np.array_equal(traj["s"], s)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    W_d = np.zeros((21, n, n), np.int64)
    np.add.at(W_d, (dly.astype(np.int64), src, tgt), 4 * wq.astype(np.int64))
    jfx = round(0.3 * 65536)
    ext = np.stack([oracle.ext_counts(p, u) for u in range(T)])
    for u in range(T):
        a = ext[u].astype(np.int64) * jfx
        for d in range(1, 21):
            if u - d >= 0:
                a += s[u - d] @ W_d[d]
        assert np.array_equal(a, traj["input"][u].astype(np.int64)), u
    c = sim.counts()
    assert c["spikes"] == s.sum()
    assert c["e_rec"] == int((s.sum(0) * np.diff(row_ptr)).sum())
    assert c["e_ext"] == int(ext.sum())


def test_conservation_of_delivered_input(tiny_run):
    p, (row_ptr, tgt, dly, wq), sim, T = tiny_run
    n = oracle.n_neurons(p)
    rowsum = np.add.reduceat(4 * wq.astype(np.int64), row_ptr[:-1]) * (np.diff(row_ptr) > 0)
    emitted = 0
    for u in range(T):
        emitted += int(rowsum[sim.spikes(u)].sum())
    jfx = round(0.3 * 65536)
    lhs = sim.consumed() + int(sim.state()["pend"].astype(np.int64).sum())
    assert lhs == emitted + jfx * sim.counts()["e_ext"]


def test_synapse_order_does_not_matter():
    p = W.tiny(2, 2, npc=40, seed=9)
    row_ptr, tgt, dly, wq = oracle.network(p)
    rng = np.random.default_rng(0)
    perm = np.concatenate([row_ptr[i] + rng.permutation(row_ptr[i + 1] - row_ptr[i])
                           for i in range(len(row_ptr) - 1)]).astype(np.int64)
    a = oracle.Sim(p, (row_ptr, tgt, dly, wq))
    b = oracle.Sim(p, (row_ptr, tgt[perm], dly[perm], wq[perm]))
    a.step(200)
    b.step(200)
    for u in range(200):
        assert np.array_equal(a.spikes(u), b.spikes(u))
    sa, sb = a.state(), b.state()
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(sa[k], sb[k])


def test_brute_force_helper_matches_consumed_and_pending_input(tiny_run):
    """The pair-by-pair brute-force input (used for spot checks of large networks) equals
    every recurrent input the simulation consumed and everything still pending at the end."""
    p, _, sim, T = tiny_run
    n = oracle.n_neurons(p)
    mask = np.zeros((T, n), np.uint8)
    for u in range(T):
        mask[u, sim.spikes(u)] = 1
    traj = sim.trajectory(T)
    jfx = np.int64(round(0.3 * 65536))
    targets = np.arange(n)
    for u in range(0, T, 7):
        rec = oracle.input_brute(p, targets, u, u - 1, mask, 0)
        ext = oracle.ext_counts(p, u).astype(np.int64) * jfx
        want = (traj["input"][u].astype(np.int64) - ext).astype(np.int32)
        assert np.array_equal(rec, want), u
    pend = sim.state()["pend"]
    for q in range(pend.shape[0]):
        assert np.array_equal(oracle.input_brute(p, targets, T + q, T - 1, mask, 0), pend[q]), q


def test_bulk_update_matches_the_simulation_step():
    p = W.tiny(2, 3, npc=40, seed=4)
    sim = oracle.Sim(p)
    for u in (0, 37, 90):
        sim.step(u - sim.now)
        st = sim.state()
        spk, v, ca, ref = oracle.update_many(p, u, st["pend"][0], st["v"], st["ca"], st["ref"])
        sim.step(1)
        after = sim.state()
        assert np.array_equal(np.flatnonzero(spk), sim.spikes(u))
        assert np.array_equal(v, after["v"]) and np.array_equal(ca, after["ca"])
        assert np.array_equal(ref, after["ref"])


def test_thread_count_does_not_change_the_oracle():
    """The oracle's loops over rows, neurons and spikes may run on several host threads; the
    network, the raster, the state and the counters are the same bits for one thread and
    for many (each row and neuron is computed on its own; the input is an integer sum)."""
    p = W.tiny(3, 3, npc=60, seed=41)
    T = 150
    before = oracle.threads()
    try:
        out = []
        for nt in (1, 4):
            oracle.set_threads(nt)
            net = oracle.network(p)
            sim = oracle.Sim(p, net)
            sim.step(T)
            out.append((net, sim.raster(0, T), sim.state(), sim.counts()))
    finally:
        oracle.set_threads(before)
    (n1, r1, s1, c1), (n4, r4, s4, c4) = out
    assert all(np.array_equal(a, b) for a, b in zip(n1, n4))
    assert all(np.array_equal(a, b) for a, b in zip(r1, r4))
    for k in ("v", "ca", "ref", "pend"):
        assert np.array_equal(s1[k], s4[k]), k
    assert c1 == c4 and c1["spikes"] > 0
