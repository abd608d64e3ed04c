"""Pins of the noise oracle against things other than itself:

- Philox4x64-10 against numpy's Philox bit generator (numpy increments the
  counter before each block, so its block n is philox(n + 1));
- the small-lambda inversion against scipy's Poisson quantile function for the
  same uniform;
- the transformed-rejection branch against the Poisson law: chi-square goodness
  of fit, mean and variance (a dropped term or a wrong constant in it skews the
  histogram far beyond these bounds);
- the noise transform: the counts' log-ratio gives back the line integral on
  average, and rays with no photons are clamped at one count.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import noise as Nz


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((7, 99), (5, 3, 2, 1)),
                                     ((2**64 - 1, 12345), (10**18, 2**63, 0, 42))])
def test_philox_matches_numpy(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    got = [int(x) for x in bg.random_raw(8)]
    c = list(ctr)
    want = []
    for _ in range(2):
        c[0] += 1                                   # no carry out of the first word in these cases
        want += Nz.philox4x64(c, key)
    assert got == want


def test_uniforms_are_open_and_centred():
    assert Nz.to_uniform(0) == 2.0 ** -54
    assert Nz.to_uniform(2**64 - 1) == 1.0 - 2.0 ** -54
    s = Nz.Stream(3, 17)
    u = np.array([s.next() for _ in range(4000)])
    assert abs(u.mean() - 0.5) < 0.02 and 0.0 < u.min() and u.max() < 1.0


@pytest.mark.parametrize("lam", [0.05, 0.7, 3.5, 9.9])
def test_inversion_is_the_poisson_quantile(lam):
    rng = np.random.Generator(np.random.PCG64(11))
    checked = 0
    for u in rng.uniform(0, 1, 400):
        q = int(stats.poisson.ppf(u, lam))
        # skip uniforms within rounding of a CDF step, where either neighbour is right
        if abs(stats.poisson.cdf(q, lam) - u) < 1e-12 or (q > 0 and abs(stats.poisson.cdf(q - 1, lam) - u) < 1e-12):
            continue
        assert Nz.poisson_inversion(lam, u) == q
        checked += 1
    assert checked > 390


@pytest.mark.parametrize("lam", [10.0, 37.5, 1000.0, 1e5])
def test_rejection_branch_follows_the_poisson_law(lam):
    n = 6000
    k = np.array([Nz.poisson_count(lam, 1234 + int(lam), e) for e in range(n)])
    sd = math.sqrt(lam)
    assert abs(k.mean() - lam) < 5 * sd / math.sqrt(n)
    assert abs(k.var() / lam - 1.0) < 5 * math.sqrt(2.0 / n)
    # chi-square over bins of about equal probability
    edges = np.unique(stats.poisson.ppf(np.linspace(0, 1, 21)[1:-1], lam).astype(int))
    idx = np.searchsorted(edges, k, side="left")
    obs = np.bincount(idx, minlength=len(edges) + 1)
    cdf = np.concatenate([[0.0], stats.poisson.cdf(edges, lam), [1.0]])
    # bin i holds k <= edges[i] and k > edges[i-1]
    exp = np.diff(cdf) * n
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert stats.chi2.sf(chi2, len(exp) - 1) > 1e-4, (chi2, obs, exp)


def test_noise_transform():
    photons, mu = 1e5, 0.02
    p = np.full(3000, 40.0)                              # lambda = 1e5 e^-0.8
    out, counts = Nz.poisson_noise(p, photons, mu, seed=5)
    lam = photons * math.exp(-mu * 40.0)
    assert abs(counts.mean() - lam) < 5 * math.sqrt(lam / p.size)
    np.testing.assert_allclose(out, -np.log(counts / photons) / mu, rtol=1e-15)
    assert abs(out.mean() - 40.0) < 5 * (1 / mu) / math.sqrt(lam * p.size)
    # no photons through: the count is clamped at one
    out0, c0 = Nz.poisson_noise(np.array([1e6]), photons, mu, seed=5)
    assert c0[0] == 0 and out0[0] == -math.log(1.0 / photons) / mu
    # deterministic in (seed, element)
    assert np.array_equal(Nz.poisson_noise(p[:50], photons, mu, seed=5)[1], counts[:50])
