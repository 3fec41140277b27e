"""Oracle pins for the Poisson record counts (the alternative to stochastic
rounding of a segment's expected records, Sec. 2.2.1):

- the sampler's exp(-x), built from IEEE basic operations only, is within one
  unit in the last place of the C library's exp over its domain;
- a single chunk (mean <= 64) is the inverse of the Poisson distribution function
  of an independent implementation (scipy) at the same uniform;
- chunked means (several Philox blocks) have Poisson mean, variance and shape;
- segment counts under the Poisson rule keep the expected total.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_04229_amd import workload as W

stats = pytest.importorskip("scipy.stats")


def test_exp_neg_within_one_ulp():
    xs = np.concatenate([np.linspace(0.0, 64.0, 20001), np.random.default_rng(1).uniform(0, 64, 20000),
                         [1e-300, 0.5 * math.log(2.0), math.log(2.0), 44.3614195558365, 63.999999]])
    for x in xs:
        got, ref = O.exp_neg(x), math.exp(-x)
        assert abs(got - ref) <= np.spacing(ref), (x, got, ref)


@pytest.mark.parametrize("mu", [0.3, 2.5, 12.0, 40.0, 64.0])
def test_single_chunk_is_the_inverse_distribution_function(mu):
    rng = np.random.default_rng(int(mu * 10))
    words = rng.integers(0, 2**32, 4000, dtype=np.uint64)
    u = words.astype(np.float64) / 4294967296.0
    got = np.array([O.poisson(mu, int(w)) for w in words])
    ref = stats.poisson.ppf(u, mu).astype(np.int64)
    # the sampler takes the smallest n with u < F(n), ppf the smallest with F(n) >= u
    tie = np.abs(stats.poisson.cdf(ref, mu) - u) < 1e-12
    assert np.array_equal(got[~tie], ref[~tie])


@pytest.mark.parametrize("mu", [64.5, 150.0, 1000.0, 7777.7])
def test_chunked_counts_are_poisson(mu):
    n = 6000
    rng = np.random.default_rng(int(mu))
    words = rng.integers(0, 2**32, n, dtype=np.uint64)
    got = np.array([O.poisson(mu, int(w), seed=5, seg_id=i) for i, w in enumerate(words)], dtype=np.float64)
    assert abs(got.mean() - mu) < 5.0 * math.sqrt(mu / n)
    # variance of a Poisson sample: var ~ mu, its standard error ~ mu sqrt(2 / n)
    assert abs(got.var(ddof=1) - mu) < 5.0 * mu * math.sqrt(2.0 / n)
    # shape: chi^2 against the Poisson probabilities over central quantile cells
    edges = np.unique(stats.poisson.ppf(np.linspace(0.02, 0.98, 13), mu))
    cells = np.concatenate([[-1], edges, [np.inf]]) + 0.5  # integer n falls in (e_i, e_i+1]
    obs = np.histogram(got, bins=cells)[0]
    cdf = stats.poisson.cdf(np.concatenate([[-1], edges]), mu)
    exp = np.diff(np.concatenate([cdf, [1.0]])) * n
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert stats.chi2.sf(chi2, len(exp) - 1) > 1e-4, (chi2, obs, exp)


def test_poisson_rule_keeps_the_expected_total():
    atm = O.Atmosphere(**W.ATMO_LAYERED)
    sh = W.make_shower(20000, seed=908, xmax=450.0, zenith_deg=20.0, beta="R")
    run = dict(transport="layered", detector="grid", spectrum="frank_tamm", bunch=1, h_obs=2200.0, seed=3)
    c0 = O.segment_counts(atm, O.make_run(**run), sh.seg)
    c1 = O.segment_counts(atm, O.make_run(**run, counts="poisson"), sh.seg)
    np.testing.assert_array_equal(c0["mu"], c1["mu"])
    ok = c1["status"] == 0
    tot = c1["mu"][ok].sum()
    assert abs(c1["n"][ok].sum() - tot) < 5.0 * math.sqrt(tot)
    # per segment the count is the sampler's draw for its mean and its own word
    assert np.std(c1["n"][ok] - c1["mu"][ok]) > np.std(c0["n"][ok] - c0["mu"][ok])
