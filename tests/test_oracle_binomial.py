"""Pins of the oracle's binomial sampler (inversion with chunking and the
p > 1/2 complement) against the textbook binomial law (scipy.stats.binom)."""
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
                                 (40, 0.97), (300, 0.25), (1500, 0.2), (2500, 0.6)])
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
