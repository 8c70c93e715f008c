"""Pins of the oracle's binomial sampler (inversion with chunking for n p < 10,
Hormann's BTRD rejection above, and the p > 1/2 complement) against the
textbook binomial law (scipy.stats.binom)."""
import numpy as np
import pytest
from scipy import stats


def _chi2_pvalue(samples, m, p):
    ks = np.arange(0, m + 1)
    pmf = stats.binom.pmf(ks, m, p)
    obs = np.bincount(samples, minlength=m + 1)[: m + 1].astype(float)
    n = samples.size
    exp = pmf * n
    # pool the tails where the expected count is small
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < 5:
        o[-2] += o[-1]; e[-2] += e[-1]; o = o[:-1]; e = e[:-1]
    chi2 = ((o - e) ** 2 / e).sum()
    return stats.chi2.sf(chi2, len(o) - 1)


@pytest.mark.parametrize("m,p", [(1, 0.3), (5, 0.3), (20, 0.05), (20, 0.5), (20, 0.7),
                                 (40, 0.97), (300, 0.25), (1500, 0.2), (2500, 0.6),
                                 (21, 0.48), (108, 0.46), (108, 0.54), (30, 0.34), (200000, 0.0007),
                                 (1000000, 0.5)])
def test_binomial_distribution(oracle_lib, m, p):
    x = oracle_lib.sample_binom(seed=99, m=m, p=p, n=40000)
    assert x.min() >= 0 and x.max() <= m
    assert _chi2_pvalue(x, m, p) > 1e-3
    se = np.sqrt(m * p * (1 - p) / x.size)
    assert abs(x.mean() - m * p) < 4 * se + 1e-12


def test_binomial_degenerate(oracle_lib):
    assert np.all(oracle_lib.sample_binom(1, m=0, p=0.5, n=100) == 0)
    assert np.all(oracle_lib.sample_binom(1, m=17, p=0.0, n=100) == 0)
    assert np.all(oracle_lib.sample_binom(1, m=17, p=1.0, n=100) == 17)
    assert np.all(oracle_lib.sample_binom(1, m=17, p=1.5, n=100) == 17)
    # p one ulp below 1: the complement Bin(m, 2^-53) is 0 for any 32-bit uniform
    assert np.all(oracle_lib.sample_binom(1, m=1000, p=1.0 - 2.0**-53, n=1000) == 1000)


def test_btrd_tails_and_branches(oracle_lib):
    """n p = 50 (the dendrite's largest items): 400,000 variates against the
    exact law, binned so that the tails beyond the squeeze (|k - mode| > 15,
    where Stirling's series decides) carry their own bins, plus the first
    four moments."""
    m, p = 108, 0.46
    x = oracle_lib.sample_binom(seed=7, m=m, p=p, n=400000, stream_id=5, window=3)
    ks = np.arange(m + 1)
    cdf = stats.binom.cdf(ks, m, p)
    mode = int((m + 1) * p)
    edges = [-1, mode - 20, mode - 16, mode - 12, mode - 8, mode - 3, mode, mode + 3, mode + 8, mode + 12,
             mode + 16, mode + 20, m]
    obs = np.histogram(x, bins=np.array(edges) + 0.5)[0]
    exp = np.diff(np.concatenate([[0.0], cdf[np.array(edges[1:])]])) * x.size
    assert exp.min() > 5
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-3
    mean, var = m * p, m * p * (1 - p)
    assert abs(x.mean() - mean) < 4 * np.sqrt(var / x.size)
    assert abs(x.var() - var) < 4 * var * np.sqrt(2.0 / x.size)
    z = (x - mean) / np.sqrt(var)
    assert abs((z ** 3).mean() - (1 - 2 * p) / np.sqrt(var)) < 0.02


def test_sqrt_newton_within_an_ulp(oracle_lib):
    rng = np.random.default_rng(3)
    xs = np.concatenate([[1.0, 2.0, 3.0, 4.0, 5.0, 2.0**52, 2.0**53 - 1, 10.0, 1e300],
                         np.exp(rng.uniform(0.0, 690.0, 20000))])
    for x in xs:
        y = oracle_lib.sqrt_newton(x)
        ref = np.sqrt(x)
        assert abs(y - ref) <= np.spacing(ref), (x, y, ref)
