"""Pins of the oracle's binomial samplers against exact pmfs (scipy.stats).

The paper draws spawn and death counts from binomial and multinomial laws and
cites BINV / BTRD-type generators (Sec. III.B).  Each case is a chi-square test
of 10^5-2*10^5 samples against the exact pmf, over a grid that covers the
inversion branch (n p < 10), the transformed-rejection branch (n p >= 10) and
its exact-recursion / squeeze / final-test sub-branches, the p > 1/2
reflection, the zero-truncated law and the integer-plus-fraction split.
"""
import numpy as np
import pytest
from scipy import stats

PTHRESH = 1e-4  # reject only on a gross mismatch; seeds are fixed


def _chi2_pvalue(samples, pmf_support, pmf):
    lo, hi = pmf_support
    ks = np.arange(lo, hi + 1)
    expected = pmf(ks) * len(samples)
    counts = np.bincount(samples - lo, minlength=len(ks))[:len(ks)]
    assert counts.sum() == len(samples), "sample outside the support"
    # pool bins with small expectation into their neighbours
    e_b, c_b = [], []
    e_acc = c_acc = 0.0
    for e, c in zip(expected, counts):
        e_acc += e
        c_acc += c
        if e_acc >= 20:
            e_b.append(e_acc)
            c_b.append(c_acc)
            e_acc = c_acc = 0.0
    if e_acc > 0:
        if e_b:
            e_b[-1] += e_acc
            c_b[-1] += c_acc
        else:
            e_b.append(e_acc)
            c_b.append(c_acc)
    e_b = np.array(e_b)
    c_b = np.array(c_b)
    if len(e_b) < 2:
        return 1.0
    chi2 = ((c_b - e_b) ** 2 / e_b).sum()
    return stats.chi2.sf(chi2, len(e_b) - 1)


BIN_CASES = [(1, 0.3), (3, 0.001), (7, 0.2), (40, 0.2), (200, 0.049), (12, 0.5),
             (30, 0.34), (100, 0.1), (1000, 0.3), (100000, 0.02), (2 ** 31 - 1, 1e-6),
             (25, 0.6), (300, 0.9), (9, 0.999)]


@pytest.mark.parametrize("n,p", BIN_CASES)
def test_binomial_pmf(orc, n, p):
    x = orc.binom_many(n, p, 0, seed=11, count=150000)
    assert x.min() >= 0 and x.max() <= n
    lo, hi = int(x.min()), int(x.max())
    pv = _chi2_pvalue(x, (lo, hi), lambda k: stats.binom.pmf(k, n, p) /
                      (stats.binom.cdf(hi, n, p) - stats.binom.cdf(lo - 1, n, p)))
    assert pv > PTHRESH
    # and the mean against n p to ~5 sigma
    assert abs(x.mean() - n * p) <= 5 * np.sqrt(n * p * (1 - p) / len(x)) + 1e-12


@pytest.mark.parametrize("n,p", [(1, 0.01), (3, 0.2), (50, 0.05), (400, 0.1), (5, 0.8),
                                 (1, 0.9), (20000, 0.001)])
def test_truncated_binomial_pmf(orc, n, p):
    x = orc.binom_many(n, p, 1, seed=12, count=120000)
    assert x.min() >= 1 and x.max() <= n
    z = 1.0 - stats.binom.pmf(0, n, p)
    hi = int(x.max())
    pv = _chi2_pvalue(x, (1, hi), lambda k: stats.binom.pmf(k, n, p) / z)
    assert pv > PTHRESH


@pytest.mark.parametrize("n,P", [(3, 2.4), (10, 1.0), (7, 0.3), (1000, 3.05)])
def test_bsplit_integer_plus_fraction(orc, n, P):
    x = orc.binom_many(n, P, 2, seed=13, count=60000)
    f = np.floor(P)
    base = n * int(f)
    frac = P - f
    assert x.min() >= base and x.max() <= base + (n if frac > 0 else 0)
    y = x - base
    if frac > 0:
        pv = _chi2_pvalue(y, (int(y.min()), int(y.max())),
                          lambda k: stats.binom.pmf(k, n, frac) /
                          (stats.binom.cdf(y.max(), n, frac) - stats.binom.cdf(y.min() - 1, n, frac)))
        assert pv > PTHRESH
    else:
        assert np.all(y == 0)


def test_binomial_degenerate(orc):
    assert np.all(orc.binom_many(0, 0.3, 0, 1, 100) == 0)
    assert np.all(orc.binom_many(17, 0.0, 0, 1, 100) == 0)
    assert np.all(orc.binom_many(17, 1.0, 0, 1, 100) == 17)


CH_CASES = [
    # probabilities of the 8 channels, counts (R parts x4, I parts x4)
    ([0.01, 0.002, 0.004, 0.03, 0.01, 0.002, 0.004, 0.03], [3] * 4 + [2] * 4),
    ([0.2, 0.0, 0.1, 0.05, 0.2, 0.0, 0.1, 0.05], [5] * 4 + [0] * 4),
    ([0.001, 0.001, 0.0, 0.008, 0.001, 0.001, 0.0, 0.008], [1500] * 4 + [40] * 4),
    ([1.3, 0.02, 0.1, 0.4, 1.3, 0.02, 0.1, 0.4], [4] * 4 + [1] * 4),  # one p >= 1
]


@pytest.mark.parametrize("p,n", CH_CASES)
def test_channel_counts_are_independent_binomials(orc, p, n):
    """The entry-level sampler (one uniform decides 'nothing happens' or the first
    nonzero channel) must give eight independent Bsplit(n_k, p_k) counts."""
    X = orc.channels_many(p, n, seed=21, count=120000)
    for k in range(8):
        x = X[:, k]
        if n[k] == 0 or p[k] == 0:
            assert np.all(x == 0)
            continue
        f = np.floor(p[k])
        frac = p[k] - f
        y = x - n[k] * int(f)
        assert y.min() >= 0
        if frac == 0:
            assert np.all(y == 0)
            continue
        lo, hi = int(y.min()), int(y.max())
        pv = _chi2_pvalue(y, (lo, hi), lambda kk: stats.binom.pmf(kk, n[k], frac) /
                          (stats.binom.cdf(hi, n[k], frac) - stats.binom.cdf(lo - 1, n[k], frac)))
        assert pv > PTHRESH, (k, pv)
    # independence: joint zero pattern of channel pairs against the product law
    zero = X == 0
    for a in range(8):
        for b in range(a + 1, 8):
            if zero[:, a].all() or zero[:, b].all() or (~zero[:, a]).all() or (~zero[:, b]).all():
                continue
            table = np.array([[np.sum(zero[:, a] & zero[:, b]), np.sum(zero[:, a] & ~zero[:, b])],
                              [np.sum(~zero[:, a] & zero[:, b]), np.sum(~zero[:, a] & ~zero[:, b])]])
            if table.min() < 5:
                continue
            pv = stats.chi2_contingency(table)[1]
            assert pv > PTHRESH, (a, b, pv)
    # the probability that nothing happens is the product of the zero probabilities
    p_none = np.prod([(1 - pk) ** nk if pk < 1 else (0.0 if nk else 1.0) for pk, nk in zip(p, n)])
    obs = np.mean(np.all(X == 0, axis=1))
    assert abs(obs - p_none) <= 5 * np.sqrt(max(p_none * (1 - p_none), 1e-12) / len(X)) + 1e-12


@pytest.mark.parametrize("p,n", CH_CASES[:3])
def test_no_event_prob_is_the_all_zero_frequency(orc, p, n):
    """The no-event probability is prod_k (1 - p_k)^n_k: against the exact power
    product (math.prod of real powers, within rounding) and against the
    frequency with which the channel sampler returns eight zero counts."""
    import math
    g = orc.no_event_prob(p, n)
    exact = math.prod((1.0 - pk) ** nk for pk, nk in zip(p, n))
    assert abs(g - exact) <= 1e-12 * exact
    X = orc.channels_many(p, n, seed=33, count=200000)
    freq = np.mean(np.all(X == 0, axis=1))
    sd = math.sqrt(g * (1 - g) / len(X))
    assert abs(freq - g) < 5 * sd + 1e-12, (freq, g)


def test_no_event_prob_special_cases(orc):
    z = [0.0] * 8
    assert orc.no_event_prob(z, [7] * 8) == 1.0
    assert orc.no_event_prob([0.3] * 8, [0] * 8) == 1.0
    # one channel: (1 - p)^n by binary powers, 0.75^4 = 0.31640625 exactly
    assert orc.no_event_prob([0.25] + [0.0] * 7, [4] + [0] * 7) == 0.31640625
    assert orc.no_event_prob([0.5] * 4 + [0.0] * 4, [3] * 4 + [9] * 4) == 2.0 ** -12
