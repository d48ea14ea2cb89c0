"""Pins of the oracle's FP64 surrogate-gradient adjoint (CPU only).

On the soft model -- the step with the spike replaced by the smooth S(x) = 1/beta +
x / (1 + beta |x|), whose derivative is exactly the surrogate -- the adjoint recursion is
the exact gradient of the loss, so central finite differences of the FP64 soft forward
check every term of it (leak, AHP, calcium, reset, delayed recurrent delivery, weights).
On the hard model the same recursion runs over the recorded spike mask; there a weight
whose source never spiked must get exactly zero gradient.  With the mask frozen and the
surrogate switched off, the hard step is smooth, and central finite differences of an
independent numpy forward check the recursion's refractory gate, reset and delayed
delivery; a one-neuron closed form pins the gate and the calcium path through refractory
steps exactly.
"""
import numpy as np
import pytest

import oracle
from paper_1511_09325_amd import workloads as W

BETA = 5.0


def _setup(T=40):
    p = W.tiny(2, 2, npc=10, seed=3, ext_rate_hz=3.2)
    net = oracle.network(p)
    w0 = net[3].astype(np.float64) / 16384.0
    n = oracle.n_neurons(p)
    targets = np.random.default_rng(0).uniform(2.0, 8.0, size=4)
    return p, net, w0, n, targets, T


def _loss_and_dlds(p, s, targets, T):
    n = s.shape[1]
    npc = p["npc"]
    scale = 1000.0 / (npc * T * p["dt"])
    rates = s.reshape(T, -1, npc).sum(axis=(0, 2)) * scale
    C = len(rates)
    loss = ((rates - targets) ** 2).sum() / C
    dr = 2.0 * (rates - targets) / C
    dl_ds = np.repeat(dr, npc)[None, :].repeat(T, 0) * scale
    return loss, dl_ds


def _soft_loss(p, net, w, targets, T):
    consts = oracle.step_constants(p, single=False)
    traj = oracle.soft_forward(p, consts, BETA, net, w, T)
    return _loss_and_dlds(p, traj["s"], targets, T)[0]


def test_soft_model_adjoint_matches_finite_differences():
    p, net, w0, n, targets, T = _setup()
    consts = oracle.step_constants(p, single=False)
    traj = oracle.soft_forward(p, consts, BETA, net, w0, T)
    loss, dl_ds = _loss_and_dlds(p, traj["s"], targets, T)
    assert np.isfinite(loss) and loss > 0
    gw, gpm, ggam = oracle.adjoint(consts, BETA, net, w0, traj, dl_ds)
    # tau_m through P_m = exp(-dt / tau_m)
    g_tau = gpm * consts["pm"] * p["dt"] / p["tau_m"] ** 2
    h = 1e-6 * p["tau_m"]
    fd = (_soft_loss(dict(p, tau_m=p["tau_m"] + h), net, w0, targets, T) -
          _soft_loss(dict(p, tau_m=p["tau_m"] - h), net, w0, targets, T)) / (2 * h)
    assert abs(fd - g_tau) <= 1e-6 * abs(fd) + 1e-12
    # g_AHP through gamma = g_AHP dt
    g_g = ggam * p["dt"]
    h = 1e-6 * p["g_ahp"]
    fd = (_soft_loss(dict(p, g_ahp=p["g_ahp"] + h), net, w0, targets, T) -
          _soft_loss(dict(p, g_ahp=p["g_ahp"] - h), net, w0, targets, T)) / (2 * h)
    assert abs(fd - g_g) <= 1e-6 * abs(fd) + 1e-12
    # 32 sampled weights
    rng = np.random.default_rng(1)
    for e in rng.choice(len(w0), size=32, replace=False):
        h = 1e-4 * max(abs(w0[e]), 1e-3)   # FD roundoff eps*L/h stays below 1e-8 relative
        wp, wm = w0.copy(), w0.copy()
        wp[e] += h
        wm[e] -= h
        fd = (_soft_loss(p, net, wp, targets, T) - _soft_loss(p, net, wm, targets, T)) / (2 * h)
        assert abs(fd - gw[e]) <= 1e-6 * max(abs(fd), 1e-9) + 1e-12, (e, fd, gw[e])


def test_hard_model_silent_source_gets_zero_gradient():
    p = W.tiny(2, 2, npc=20, seed=8)
    net = oracle.network(p)
    T = 60
    sim = oracle.Sim(p, net)
    sim.record(True)
    sim.step(T)
    tr = sim.trajectory(T)
    traj = {"v_prev": tr["v_prev"], "ca_prev": tr["ca_prev"], "v_tilde": tr["v_tilde"],
            "s": tr["s"].astype(np.float64), "r": tr["r"]}
    consts = oracle.step_constants(p, single=True)
    targets = np.full(4, 5.0)
    _, dl_ds = _loss_and_dlds(p, traj["s"], targets, T)
    w = net[3].astype(np.float64) / 16384.0
    gw, gpm, ggam = oracle.adjoint(consts, BETA, net, w, traj, dl_ds)
    fired = traj["s"].sum(0) > 0
    src = np.repeat(np.arange(len(net[0]) - 1), np.diff(net[0]))
    assert fired.any() and (~fired).any()
    assert np.all(gw[~fired[src]] == 0.0)
    assert np.any(gw[fired[src]] != 0.0)
    assert np.isfinite(gpm) and np.isfinite(ggam)


# ---- hard model with the spike mask frozen ---------------------------------------------------
#
# With the spikes s(u) and refractory flags r(u) of a hard run held fixed, the step is smooth
# (linear in the weights): refractory steps hold V at V_reset and ignore V(u-1) and the input,
# a spike resets V to V_reset, calcium decays every step and jumps by alpha at spikes.  A loss
# L = sum over non-refractory (u, j) of c[u, j] V~_j(u) then has an exact gradient, which the
# adjoint recursion gives with the surrogate switched off (sigma' = 0, beta -> infinity) and
# dL/dV~ = c entering directly.  The masked forward below is written from that description
# in plain numpy, independently of the oracle's C code.

BETA_OFF = 1e300   # sigma'(x) = 1 / (1 + beta |x|)^2 underflows to 0 for any x != 0


def _masked_setup(T=40):
    p = W.tiny(2, 2, npc=10, seed=3, ext_rate_hz=3.4)
    net = oracle.network(p)
    sim = oracle.Sim(p, net)
    sim.record(True)
    sim.step(T)
    tr = sim.trajectory(T)
    n = oracle.n_neurons(p)
    ext = np.stack([oracle.ext_counts(p, u) for u in range(T)]).astype(np.float64)
    jext = np.rint(p["j_ext"] * 65536.0) / 65536.0
    v0 = np.array([oracle.initial_v(p, j) for j in range(n)], np.float64)
    c = np.random.default_rng(9).normal(size=(T, n)) * (1 - tr["r"])
    return p, net, tr, ext * jext, v0, c


def _masked_loss(p, net, w, pm, gam, pc, tr, ext_mv, v0, c):
    row_ptr, tgt, dly = net[0], net[1], net[2]
    T, n = tr["s"].shape
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    s = tr["s"].astype(np.float64)
    r = tr["r"].astype(bool)
    v, ca = v0.copy(), np.zeros(n)
    loss = 0.0
    for u in range(T):
        cur = ext_mv[u].copy()
        e = u - dly.astype(np.int64)
        ok = e >= 0
        np.add.at(cur, tgt[ok], w[ok] * s[e[ok], src[ok]])
        vt = pm * v - gam * ca + cur
        loss += float((c[u] * np.where(r[u], 0.0, vt)).sum())
        v = np.where(r[u] | (s[u] > 0), p["v_reset"], vt)
        ca = pc * ca + p["ca_inc"] * s[u]
    return loss


def test_frozen_mask_adjoint_matches_finite_differences():
    T = 40
    p, net, tr, ext_mv, v0, c = _masked_setup(T)
    assert tr["s"].sum() > 0 and tr["r"].sum() > 0
    consts = oracle.step_constants(p, single=False)
    pm, gam, pc = consts["pm"], consts["gamma"], consts["pc"]
    w0 = net[3].astype(np.float64) / 16384.0
    # the trajectory the adjoint needs, from the masked forward itself (FP64)
    n = len(v0)
    vp, cp, vts = np.zeros((T, n)), np.zeros((T, n)), np.zeros((T, n))
    v, ca = v0.copy(), np.zeros(n)
    s, r = tr["s"].astype(np.float64), tr["r"].astype(bool)
    src = np.repeat(np.arange(n), np.diff(net[0]))
    for u in range(T):
        cur = ext_mv[u].copy()
        e = u - net[2].astype(np.int64)
        ok = e >= 0
        np.add.at(cur, net[1][ok], w0[ok] * s[e[ok], src[ok]])
        vt = pm * v - gam * ca + cur
        vp[u], cp[u], vts[u] = v, ca, np.where(r[u], 0.0, vt)
        v = np.where(r[u] | (s[u] > 0), p["v_reset"], vt)
        ca = pc * ca + p["ca_inc"] * s[u]
    traj = {"v_prev": vp, "ca_prev": cp, "v_tilde": vts, "s": s, "r": tr["r"]}
    gw, gpm, ggam = oracle.adjoint(consts, BETA_OFF, net, w0, traj, np.zeros((T, n)), dl_dvt=c)
    L = lambda w=w0, pm_=pm, g_=gam: _masked_loss(p, net, w, pm_, g_, pc, tr, ext_mv, v0, c)
    h = 1e-6
    fd_pm = (L(pm_=pm + h) - L(pm_=pm - h)) / (2 * h)
    fd_g = (L(g_=gam + h) - L(g_=gam - h)) / (2 * h)
    assert abs(fd_pm - gpm) <= 1e-6 * abs(fd_pm), (fd_pm, gpm)
    assert abs(fd_g - ggam) <= 1e-6 * abs(fd_g), (fd_g, ggam)
    rng = np.random.default_rng(2)
    fired = tr["s"].sum(0) > 0
    live = np.flatnonzero(fired[src])
    for e in rng.choice(live, size=32, replace=False):
        wp, wm = w0.copy(), w0.copy()
        wp[e] += 1e-3
        wm[e] -= 1e-3
        fd = (L(w=wp) - L(w=wm)) / 2e-3   # the loss is linear in each weight: exact
        assert abs(fd - gw[e]) <= 1e-9 * max(abs(fd), 1.0), (e, fd, gw[e])


def _single_neuron(s, r, v_tilde, dl_dvt, beta, probe):
    """The adjoint of one neuron with no synapses; returns nu(probe), read out through
    dL/dP_m = sum_u V(u-1) nu(u) with V(u-1) the indicator of step `probe`."""
    T = len(s)
    consts = dict(pm=0.95, pc=0.99, gamma=0.2, alpha=0.05, theta=20.0, vreset=15.0)
    net = (np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint8))
    col = lambda x: np.asarray(x, np.float64).reshape(T, 1)
    traj = {"v_prev": col(np.arange(T) == probe), "ca_prev": col(np.zeros(T)),
            "v_tilde": col(v_tilde), "s": col(s), "r": np.asarray(r, np.uint8).reshape(T, 1)}
    _, gpm, _ = oracle.adjoint(consts, beta, net, np.zeros(0), traj, col(np.zeros(T)),
                               dl_dvt=col(dl_dvt))
    return gpm, consts


def test_refractory_steps_block_the_gradient_closed_form():
    """One neuron spikes at step 1 and is refractory at steps 2 and 3 (two steps, V held at
    V_reset).  With the surrogate off, a loss on V~(4) reaches back only to step 4: nothing
    passes the clamped steps, whatever direct gradient they carry (7 here), and the spike's
    reset cuts V~(1) from V(1).  With the surrogate on, the only path from step 4 to step 1
    is calcium: mu(3) = -gamma nu(4), carried over the refractory steps by P_c alone, so
    nu(1) = alpha (-gamma P_c^2 nu(4)) sigma'(V~(1) - theta)."""
    s, r = [0, 1, 0, 0, 0], [0, 0, 1, 1, 0]
    vt = [18.0, 21.0, 0.0, 0.0, 19.0]
    dl = [0.0, 0.0, 7.0, 7.0, 1.0]
    nu = [_single_neuron(s, r, vt, dl, BETA_OFF, u)[0] for u in range(5)]
    assert nu == [0.0, 0.0, 0.0, 0.0, 1.0]
    nu1, k = _single_neuron(s, r, vt, dl, BETA, 1)
    nu4, _ = _single_neuron(s, r, vt, dl, BETA, 4)
    assert nu4 == 1.0  # lambda(4) = mu(4) = 0, so e(4) = 0 and nu(4) is the direct term
    sig1 = 1.0 / (1.0 + BETA * abs(vt[1] - k["theta"])) ** 2
    want = k["alpha"] * (-k["gamma"] * k["pc"] ** 2 * nu4) * sig1
    assert abs(nu1 - want) <= 1e-15 * abs(want), (nu1, want)
    for u in (2, 3):
        assert _single_neuron(s, r, vt, dl, BETA, u)[0] == 0.0
