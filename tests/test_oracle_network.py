"""Pins of the oracle's network generator (CPU only).

The generator follows the paper's network description (section 2, Methods; Table 1):
columns of 1240 point neurons (80 % excitatory) on a 2-D grid, most synapses inside the
own column and the rest to neighbouring columns with a probability falling with
distance, about 1240 synapses per neuron.  These tests check it against what that
description and the workload recipe fix: the printed problem sizes, the expected
out-degree, the own-column share, the neighbour split, uniform delays, the weight
moments, and an independent numpy re-derivation of individual rows.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1511_09325_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    for line in open(os.path.join(GOLDEN, "paper_table1.txt")):
        if line.startswith("#") or not line.strip():
            continue
        g, cols, neu, rec, tot = line.split()
        rows.append((int(g), int(cols), float(neu), float(rec), float(tot)))
    return rows


def test_table1_problem_sizes():
    """Neurons and expected synapses of the three grids agree with the paper's Table 1."""
    for g, ncols, neu_m, rec_g, tot_g in _table1():
        p = W.grid(g, g)
        assert p["rows"] * p["cols"] == ncols
        n = oracle.n_neurons(p)
        assert abs(n / 1e6 - neu_m) / neu_m < 0.03
        # expected out-degree: every column pair's probability summed over the stencil is 1,
        # minus the excluded self pair in the own column
        deg = p["npc"] * (p["p_own"] + p["p_remote"]) - p["p_own"]
        assert abs(deg - 1239.4) < 1e-9
        assert abs(deg * n / 1e9 - rec_g) / rec_g < 0.03
        assert abs((deg + 540) * n / 1e9 - tot_g) / tot_g < 0.06


def test_neighbour_probabilities():
    p = W.grid(5, 5)
    e1, e2 = math.exp(-1.0), math.exp(-math.sqrt(2.0))
    pe = 0.4 * e1 / (4 * e1 + 4 * e2)
    pd = 0.4 * e2 / (4 * e1 + 4 * e2)
    assert abs(pe - 0.0602098) < 1e-7 and abs(pd - 0.0397902) < 1e-7
    c = 2 * 5 + 2
    assert oracle.column_probability(p, c, c) == 0.6
    assert abs(oracle.column_probability(p, c, c + 1) - pe) < 1e-15
    assert abs(oracle.column_probability(p, c, c + 6) - pd) < 1e-15
    assert oracle.column_probability(p, c, c + 2) == 0.0
    # periodic wrap: column (0,0) reaches (4,4) diagonally
    assert abs(oracle.column_probability(p, 0, 24) - pd) < 1e-15
    # on a 2x2 torus opposite offsets land on the same column and add up
    q = W.grid(2, 2)
    assert abs(oracle.column_probability(q, 0, 1) - 2 * pe) < 1e-15
    assert abs(oracle.column_probability(q, 0, 3) - 4 * pd) < 1e-15
    for g in [(2, 2), (2, 5), (5, 3), (1, 1), (3, 3)]:
        r = W.grid(*g)
        total = sum(oracle.column_probability(r, 0, t) for t in range(g[0] * g[1]))
        assert abs(total - 1.0) < 1e-12


@pytest.fixture(scope="module")
def net2x2():
    p = W.grid(2, 2, 0)
    return p, oracle.network(p)


def test_rows_sorted_no_self_no_multapse(net2x2):
    p, (row_ptr, tgt, dly, wq) = net2x2
    n = oracle.n_neurons(p)
    for i in range(0, n, 97):
        a, b = row_ptr[i], row_ptr[i + 1]
        key = dly[a:b].astype(np.int64) * (1 << 32) + tgt[a:b]
        assert np.all(np.diff(key) > 0)         # sorted by (delay, target), no duplicates
        assert not np.any(tgt[a:b] == i)


def test_out_degree_and_own_column_share(net2x2):
    p, (row_ptr, tgt, dly, wq) = net2x2
    n = oracle.n_neurons(p)
    deg = np.diff(row_ptr)
    assert len(tgt) == row_ptr[-1]
    # "~6.15M" synapses for the 2x2 grid; expected 1239.4 per neuron
    assert abs(deg.mean() - 1239.4) < 4 * deg.std() / np.sqrt(n)
    src_col = np.repeat(np.arange(n) // p["npc"], deg)
    tgt_col = tgt // p["npc"]
    own = np.bincount(np.repeat(np.arange(n), deg)[src_col == tgt_col], minlength=n)
    exp_own = 0.6 * 1239
    assert abs(own.mean() - exp_own) < 4 * np.sqrt(1239 * 0.6 * 0.4 / n)
    # 2x2: each other column receives 1240 * (summed probability)
    for other, prob in [(1, 2 * 0.0602098), (2, 2 * 0.0602098), (3, 4 * 0.0397902)]:
        m = ((src_col == 0) & (tgt_col == other)).sum() / p["npc"]
        assert abs(m - 1240 * prob) < 4 * np.sqrt(1240 * prob / p["npc"])


def test_delays_uniform(net2x2):
    p, (row_ptr, tgt, dly, wq) = net2x2
    assert dly.min() == 1 and dly.max() == 20
    obs = np.bincount(dly, minlength=21)[1:]
    chi2, pval = stats.chisquare(obs)
    assert pval > 1e-4


def test_weight_moments(net2x2):
    p, (row_ptr, tgt, dly, wq) = net2x2
    n = oracle.n_neurons(p)
    deg = np.diff(row_ptr)
    exc = np.repeat((np.arange(n) % p["npc"]) < p["n_exc"], deg)
    for mask, mu, sd in [(exc, 0.2, 0.02), (~exc, -0.8, 0.08)]:
        w = wq[mask].astype(np.float64) / 16384.0
        assert abs(w.mean() - mu) < 4 * sd / np.sqrt(w.size) + 2**-15
        assert abs(w.std() / sd - 1.0) < 0.01
        assert abs(w - mu).max() <= 6 * sd + 2**-14     # Irwin-Hall(12) is bounded at 6 sigma
        # normal shape: the 1 and 2 sigma mass
        z = (w - mu) / sd
        assert abs((np.abs(z) < 1).mean() - 0.6827) < 0.01
        assert abs((np.abs(z) < 2).mean() - 0.9545) < 0.005
    assert np.all(wq[exc] > 0) and np.all(wq[~exc] < 0)


# ---- an independent numpy derivation of single rows from the published Philox -----------
_M0, _M1, _W0, _W1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57), 0x9E3779B9, 0xBB67AE85


def _philox_np(c0, c1, c2, c3, key):
    m32 = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, np.uint64) for x in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & m32, p1 & m32,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & m32, p0 & m32]
        k0 = np.uint64((int(k0) + _W0) & 0xFFFFFFFF)
        k1 = np.uint64((int(k1) + _W1) & 0xFFFFFFFF)
    return c


def _row_np(p, i):
    npc, ncol = p["npc"], p["rows"] * p["cols"]
    key = (p["seed"] & 0xFFFFFFFF, p["seed"] >> 32)
    j = np.arange(ncol * npc, dtype=np.uint64)
    thr = np.array([math.floor(oracle.column_probability(p, i // npc, c) * 2**32)
                    for c in range(ncol)], dtype=np.float64)
    thr = np.repeat(np.minimum(thr, 2**32), npc)
    r = _philox_np(j, np.full_like(j, i), np.zeros_like(j), np.full_like(j, 1), key)
    conn = (r[0].astype(np.float64) < thr) & (j != i)
    d = 1 + ((r[1] * np.uint64(20)) >> np.uint64(32)).astype(np.int64)
    r2 = _philox_np(j, np.full_like(j, i), np.ones_like(j), np.full_like(j, 1), key)
    s = np.zeros(j.shape, np.int64)
    for wd in (r[2], r[3], r2[0], r2[1], r2[2], r2[3]):
        s += (wd & np.uint64(0xFFFF)).astype(np.int64) + (wd >> np.uint64(16)).astype(np.int64)
    z = (s - 393210).astype(np.float64) / 65536.0
    exc = (i % npc) < p["n_exc"]
    mu, sd = (0.2, 0.02) if exc else (-0.8, 0.08)
    w = np.rint((mu + sd * z) * 16384.0).astype(np.int16)
    sel = np.nonzero(conn)[0]
    order = np.lexsort((sel, d[sel]))
    sel = sel[order]
    return sel.astype(np.int32), d[sel].astype(np.uint8), w[sel]


@pytest.mark.parametrize("shape,seed,rows", [((2, 2), 0, [0, 991, 992, 4959]),
                                             ((3, 4), 11, [0, 5000, 14879])])
def test_rows_match_independent_numpy_derivation(shape, seed, rows):
    p = W.grid(*shape, seed)
    for i in rows:
        t, d, w = oracle.row(p, i)
        t2, d2, w2 = _row_np(p, i)
        assert np.array_equal(t, t2) and np.array_equal(d, d2) and np.array_equal(w, w2)


def test_out_degree_independent_of_grid_shape():
    """Summed-probability wrap keeps the expected out-degree at 1239.4 on every torus."""
    for shape in [(2, 5), (5, 3), (3, 3)]:
        p = W.grid(*shape, 3)
        n = oracle.n_neurons(p)
        degs = [len(oracle.row(p, i)[0]) for i in range(0, n, max(1, n // 60))]
        assert abs(np.mean(degs) - 1239.4) < 4 * 27.7 / np.sqrt(len(degs))
