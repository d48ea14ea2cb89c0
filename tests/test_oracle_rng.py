"""Pins of the oracle's random-number building blocks (CPU only).

* Philox4x32-10 against the published known-answer vectors and against rocRAND's own
  host-side engine (an independent implementation) on random counters and keys.
* The Poisson inverse-CDF table against scipy's Poisson CDF, and the external-input
  counts' mean, variance and histogram against the Poisson law they must follow
  (external synapses as extra excitatory Poisson input, paper section 2).
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(oracle.philox(ctr, key)) == want


_ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long ctr = ((unsigned long long)c1 << 32) | c0;
    rocrand_device::philox4x32_10_engine e(seed, sub, 0);
    for (int q = 0; q < 4; ++q) e.discard(ctr);   /* 4 draws per counter step */
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
}
"""


def test_philox_matches_rocrand_engine():
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr):
        pytest.skip("rocRAND headers not installed")
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "rr.cpp")
        exe = os.path.join(td, "rr")
        open(src, "w").write(_ROCRAND_SRC)
        subprocess.check_call(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                               src, "-o", exe])
        rng = np.random.default_rng(7)
        words = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
        words[:10, :4] = 0          # include small counters
        words[10:20] = 2**32 - 1    # and all-ones
        text = "\n".join(" ".join("%x" % w for w in r) for r in words)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        got = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(words)
    for r, want in zip(words, got):
        assert list(oracle.philox(r[:4], r[4:6])) == want


@pytest.mark.parametrize("lam", [0.0, 2.0, 3.0, 4.5, 6.0])
def test_poisson_table_is_the_poisson_cdf(lam):
    tab = oracle.poisson_table(lam).astype(np.float64)
    k = np.arange(63)
    want = np.minimum(np.floor(stats.poisson.cdf(k, lam) * 2.0**32), 2.0**32) if lam > 0 \
        else np.full(63, 2.0**32)
    # the table is a floor of a CDF summed in double: within one unit of the exact floor
    assert np.all(np.abs(tab - want) <= 1.0)
    assert np.all(np.diff(tab) >= 0)


def test_poisson_count_definition_edges():
    tab = oracle.poisson_table(3.0)
    assert oracle.poisson_count(tab, 0) == 0
    t0 = int(tab[0])
    assert oracle.poisson_count(tab, t0 - 1) == 0
    assert oracle.poisson_count(tab, t0) == 1
    # lambda = 0 never draws an event, not even for the largest uniform
    z = oracle.poisson_table(0.0)
    assert oracle.poisson_count(z, 2**32 - 1) == 0


def test_external_counts_follow_poisson():
    p = dict(__import__("paper_1511_09325_amd.workloads", fromlist=["grid"]).grid(2, 2, 5))
    lam = p["ext_syn"] * p["ext_rate_hz"] * p["dt"] * 1e-3
    draws = np.concatenate([oracle.ext_counts(p, u) for u in range(200)])   # 992,000 draws
    m = draws.size
    se_mean = np.sqrt(lam / m)
    assert abs(draws.mean() - lam) < 4 * se_mean
    # variance of the sample variance of a Poisson: (mu4 - sigma^4)/m, mu4 = lam(1+3lam)
    se_var = np.sqrt((lam * (1 + 3 * lam) - lam**2) / m)
    assert abs(draws.var() - lam) < 4 * se_var
    kmax = 12
    obs = np.bincount(np.minimum(draws, kmax), minlength=kmax + 1)
    exp = stats.poisson.pmf(np.arange(kmax + 1), lam) * m
    exp[kmax] = stats.poisson.sf(kmax - 1, lam) * m
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, kmax) > 1e-4


def test_external_counts_of_one_block_are_independent():
    """Four consecutive neurons share a Philox block (one word each): their counts over many
    steps must be uncorrelated, and neighbours across block boundaries too."""
    p = dict(__import__("paper_1511_09325_amd.workloads", fromlist=["grid"]).grid(1, 1, 7))
    T = 4000
    draws = np.stack([oracle.ext_counts(p, u, 0, 8) for u in range(T)]).astype(np.float64)
    c = np.corrcoef(draws.T)
    bound = 4.0 / np.sqrt(T)
    for i in range(8):
        for j in range(i + 1, 8):
            assert abs(c[i, j]) < bound, (i, j, c[i, j])
