"""Pins of the oracle's neuron-model variants (CPU only).

The paper's neurons adapt through calcium- and sodium-dependent after-hyperpolarisation
currents (section 2), and its earlier report used Izhikevich regular-spiking (RS) and
fast-spiking (FS) neurons.  Neither variant's equations or parameters are printed in the
paper; the readings are a second AHP variable of the same form as calcium, and Izhikevich's
published model and RS/FS parameters (Izhikevich, IEEE TNN 2003).  They are pinned by what
mathematics fixes:
  * second AHP variable: its closed form under forced spikes; swapping the roles of the two
    variables leaves the run bit for bit unchanged; adaptation grows with both;
  * Izhikevich: the resting state is the stable root of 0.04 v^2 + (5 - b) v + 140 + I = 0
    (a fixed point of the dynamics with u = b v); the saddle-node at I = ((5 - b)^2 / 0.16)
    - 140 (= 4 for b = 0.2) separates rest from tonic firing; a spike resets v to c exactly
    and raises u by at least d; RS neurons adapt, and FS neurons fire faster at the same
    drive; network input is conserved whatever the neuron model.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import workloads as W

U = 2.0**-16


def _silent(n=8, **kw):
    p = W.tiny(1, 1, npc=n, p_own=0.0, p_remote=0.0, ext_rate_hz=0.0)
    p.update(kw)
    return p


def _empty_net(n):
    return (np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint8),
            np.zeros(0, np.int16))


# ---- second (sodium-dependent) AHP variable --------------------------------------------------
def test_sodium_ahp_closed_form_under_forced_spikes():
    """Na(u) = sum_k alpha_Na exp(-(u - t_k) / tau_Na) after the step, for spikes t_k forced
    by large inputs (refractory steps discard their input, as for calcium)."""
    p = _silent(n=2, g_na=0.1, tau_na=80.0, na_inc=0.03)
    sim = oracle.Sim(p, _empty_net(2))
    z = np.zeros(2)
    sim.set_state(0, z, z, z, np.zeros((21, 2), np.int32), na=z)
    forced = [2, 3, 9, 30, 31, 33, 120]
    expect = [2, 9, 30, 33, 120]
    got = []
    for u in range(260):
        if u in forced:
            sim.inject(0, 0, 100 * 65536)
        sim.step(1)
        if 0 in set(sim.spikes(u).tolist()):
            got.append(u)
        na = float(sim.state()["na"][0])
        want = sum(0.03 * math.exp(-(u - t) / 80.0) for t in expect if t <= u)
        assert abs(na - want) < 1e-6, (u, na, want)
    assert got == expect


def test_swapping_the_two_ahp_variables_changes_nothing():
    """A network whose adaptation is carried by the sodium variable (g_AHP = 0) with
    calcium's constants runs bit for bit like the calcium-only network: the second variable
    has the same form and enters V~ after the first."""
    base = W.tiny(2, 2, npc=30, seed=5, ext_rate_hz=3.4)
    a = oracle.Sim(dict(base, na_inc=0.0))
    b = oracle.Sim(dict(base, g_ahp=0.0, ca_inc=0.0, g_na=base["g_ahp"], tau_na=base["tau_ca"],
                        na_inc=base["ca_inc"]))
    a.step(200)
    b.step(200)
    assert all(np.array_equal(x, y) for x, y in zip(a.raster(0, 200), b.raster(0, 200)))
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["v"], sb["v"]) and np.array_equal(sa["pend"], sb["pend"])
    assert np.array_equal(sa["ca"], sb["na"]) and not sb["ca"].any() and not sa["na"].any()
    assert a.counts()["spikes"] > 0


def test_two_ahp_variables_adapt_more():
    """Under the same constant drive, adding the sodium AHP fires fewer spikes and ends with
    longer intervals; the one-variable sequence never shortens (a single adaptation time
    constant), and with two both ends of the sequence show adaptation."""
    def isis(**kw):
        p = _silent(n=2, **kw)
        sim = oracle.Sim(p, _empty_net(2))
        z = np.zeros(2)
        sim.set_state(0, z, z, z, np.zeros((21, 2), np.int32), na=z)
        spikes = []
        for u in range(1500):
            sim.inject(0, 0, 85_197)
            sim.step(1)
            if 0 in set(sim.spikes(u).tolist()):
                spikes.append(u)
        return np.diff(spikes)
    one = isis()
    two = isis(g_na=0.3, tau_na=100.0, na_inc=0.02)
    assert np.all(np.diff(one) >= 0) and one[-1] > one[0]
    assert two[0] < two[-20:].min()
    assert len(two) < len(one) and two[-20:].mean() > one[-20:].mean()


# ---- Izhikevich neurons ----------------------------------------------------------------------
IZH = dict(neuron_model=oracle.NEURON_IZHIKEVICH)


def _rest_root(b, current):
    """Stable fixed point of v' = 0.04 v^2 + 5 v + 140 - u + I with u = b v."""
    c1 = 5.0 - b
    disc = c1 * c1 - 0.16 * (140.0 + current)
    return (-c1 - math.sqrt(disc)) / 0.08 if disc >= 0 else None


def _izh_run(p, j, current_mv, steps, v0=None, u0=None):
    """One neuron of type j under a constant input; returns (spike steps, v, u) with v, u the
    trajectories after every step."""
    a = int(round(current_mv * 65536))
    assert a * U == current_mv
    spikes, vs, us = [], [], []
    v, u = oracle.initial_state(p, j)
    if v0 is not None:
        v, u = np.float32(v0), np.float32(u0)
    for t in range(steps):
        s, v, u, _, _ = oracle.neuron_update(p, j, t, a, float(v), float(u), 0)
        if s:
            spikes.append(t)
        vs.append(v)
        us.append(u)
    return spikes, np.array(vs, np.float64), np.array(us, np.float64)


@pytest.mark.parametrize("j", [0, 7], ids=["RS", "FS"])
def test_izhikevich_rest_is_the_stable_root(j):
    p = _silent(n=8, n_exc=4, **IZH)
    b = p["izh_b_e"] if j < 4 else p["izh_b_i"]
    for current in (0.0, 3.5):
        spikes, v, u = _izh_run(p, j, current, 2000)
        assert spikes == []
        want = _rest_root(b, current)
        assert abs(v[-1] - want) < 1e-3, (current, v[-1], want)
        assert abs(u[-1] - b * want) < 1e-3


def test_izhikevich_saddle_node_separates_rest_and_firing():
    """For b = 0.2 the resting state exists for I < 4 and vanishes above (the two roots of
    0.04 v^2 + 4.8 v + 140 + I merge at I = 4).  Below, a neuron placed at the stable root
    stays there; above, with no fixed point left, a neuron started from the same place must
    fire, and keeps firing."""
    p = _silent(n=8, n_exc=4, **IZH)
    assert _rest_root(0.2, 3.75) is not None and _rest_root(0.2, 4.25) is None
    v_rest = _rest_root(0.2, 3.75)
    for j in (0, 7):
        below, v, _ = _izh_run(p, j, 3.75, 3000, v0=v_rest, u0=0.2 * v_rest)
        above, _, _ = _izh_run(p, j, 4.25, 3000, v0=v_rest, u0=0.2 * v_rest)
        assert below == [] and abs(v[-1] - v_rest) < 1e-3
        assert len(above) >= 3 and above[-1] > 2000


def test_izhikevich_reset_and_rs_fs_signatures():
    """At I = 10: every spike leaves v at c exactly and raises u by at least
    d + a (b v_peak - u) (the recovery update uses the potential past the cut-off, then the
    reset adds d); the RS neuron's first interval is its shortest (adaptation through its
    large d); the FS neuron (fast recovery a, small d) fires more spikes than the RS one."""
    p = _silent(n=8, n_exc=4, **IZH)
    out = {}
    for j, name in ((0, "RS"), (7, "FS")):
        spikes, v, u = _izh_run(p, j, 10.0, 1000)
        sfx = "e" if j < 4 else "i"
        a, b, c, d = (p["izh_%s_%s" % (x, sfx)] for x in "abcd")
        assert len(spikes) > 5 and spikes[0] > 0
        assert np.all(v[spikes] == np.float32(c))
        before = u[np.array(spikes) - 1]
        assert np.all(u[spikes] - before >= d + a * (b * p["izh_vpeak"] - before) - 1e-4)
        out[name] = np.diff(spikes)
    rs, fs = out["RS"], out["FS"]
    assert rs[0] < rs[1:].min()
    assert len(fs) > len(rs)


def test_izhikevich_network_input_is_conserved():
    """A small Izhikevich network (RS/FS by type) fires, and every input it consumed plus
    what is still pending equals the sum over its spikes' synapses plus the external input:
    the delivery does not depend on the neuron model."""
    p = W.tiny(2, 2, npc=30, seed=7, ext_rate_hz=3.4, j_ext=1.6, **IZH)
    net = oracle.network(p)
    sim = oracle.Sim(p, net)
    T = 300
    sim.step(T)
    c = sim.counts()
    assert c["spikes"] > 0
    n = oracle.n_neurons(p)
    exc = (np.arange(n) % p["npc"]) < p["n_exc"]
    fired = set()
    for u in range(T):
        fired.update(sim.spikes(u).tolist())
    assert any(exc[list(fired)]) and any(~exc[list(fired)])
    w32 = net[3].astype(np.int64) * 4
    delivered = sum(int(w32[net[0][i]:net[0][i + 1]].sum()) for u in range(T)
                    for i in sim.spikes(u))
    ext = sum(int(oracle.ext_counts(p, u).astype(np.int64).sum()) for u in range(T))
    jfx = int(round(p["j_ext"] * 65536))
    pend = int(sim.state()["pend"].astype(np.int64).sum())
    assert sim.consumed() + pend == delivered + ext * jfx
