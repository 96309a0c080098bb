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


def _chi2_pvalue(samples, support, core, pmf, cdf):
    """Chi-square p-value of integer samples against a law on the full support
    [support[0], support[1]]: one bin per value of the core range [a, b] (where
    all but ~1e-10 of the mass lies) and one bin for each tail, whose
    expectations come from the exact cdf, so that too many (or any impossible)
    tail values count.  cdf(k) = P(X <= k) of the law itself (normalised on its
    support).  Bins with small expectation are pooled with their neighbours."""
    lo, hi = support
    a, b = max(core[0], lo), min(core[1], hi)
    x = np.asarray(samples)
    assert x.min() >= lo and x.max() <= hi, "sample outside the support"
    ks = np.arange(a, b + 1)
    expected = np.concatenate([[cdf(a - 1) if a > lo else 0.0], pmf(ks),
                               [1.0 - cdf(b) if b < hi else 0.0]]) * len(x)
    counts = np.concatenate([[np.sum(x < a)],
                             np.bincount(x[(x >= a) & (x <= b)] - a, minlength=len(ks))[:len(ks)],
                             [np.sum(x > b)]])
    assert abs(expected.sum() - len(x)) < 1e-6 * len(x), "the law's mass is not 1"
    e_b, c_b = [], []
    e_acc = c_acc = 0.0
    for e, c in zip(expected, counts):
        e_acc += e
        c_acc += c
        if e_acc >= 20:
            e_b.append(e_acc)
            c_b.append(c_acc)
            e_acc = c_acc = 0.0
    if e_acc > 0 or c_acc > 0:
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


def _binom_core(n, p):
    return int(stats.binom.ppf(1e-10, n, p)), int(stats.binom.isf(1e-10, n, p))


BIN_CASES = [(1, 0.3), (3, 0.001), (7, 0.2), (40, 0.2), (200, 0.049), (12, 0.5),
             (30, 0.34), (100, 0.1), (1000, 0.3), (100000, 0.02), (2 ** 31 - 1, 1e-6),
             (25, 0.6), (300, 0.9), (9, 0.999)]


@pytest.mark.parametrize("n,p", BIN_CASES)
def test_binomial_pmf(orc, n, p):
    x = orc.binom_many(n, p, 0, seed=11, count=150000)
    assert x.min() >= 0 and x.max() <= n
    pv = _chi2_pvalue(x, (0, n), _binom_core(n, p), lambda k: stats.binom.pmf(k, n, p),
                      lambda k: stats.binom.cdf(k, n, p))
    assert pv > PTHRESH
    # and the mean against n p to ~5 sigma
    assert abs(x.mean() - n * p) <= 5 * np.sqrt(n * p * (1 - p) / len(x)) + 1e-12


@pytest.mark.parametrize("n,p", [(1, 0.01), (3, 0.2), (50, 0.05), (400, 0.1), (5, 0.8),
                                 (1, 0.9), (20000, 0.001)])
def test_truncated_binomial_pmf(orc, n, p):
    x = orc.binom_many(n, p, 1, seed=12, count=120000)
    assert x.min() >= 1 and x.max() <= n
    z = 1.0 - stats.binom.pmf(0, n, p)
    a, b = _binom_core(n, p)
    pv = _chi2_pvalue(x, (1, n), (max(a, 1), max(b, 1)), lambda k: stats.binom.pmf(k, n, p) / z,
                      lambda k: (stats.binom.cdf(k, n, p) - stats.binom.pmf(0, n, p)) / z)
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
        pv = _chi2_pvalue(y, (0, n), _binom_core(n, frac), lambda k: stats.binom.pmf(k, n, frac),
                          lambda k: stats.binom.cdf(k, n, frac))
        assert pv > PTHRESH
    else:
        assert np.all(y == 0)


def test_chi2_sees_a_tail_error():
    """The full-support chi-square has teeth in the tails: a sampler that is
    right in the core but puts 0.5% of its draws far in the right tail fails,
    which the former range-normalised test (the pmf renormalised over the
    observed min..max) could not see."""
    rng = np.random.default_rng(5)
    n, p = 1000, 0.3
    good = rng.binomial(n, p, 150000)
    core = _binom_core(n, p)
    law = (lambda k: stats.binom.pmf(k, n, p), lambda k: stats.binom.cdf(k, n, p))
    assert _chi2_pvalue(good, (0, n), core, *law) > PTHRESH
    bad = good.copy()
    bad[:750] = rng.integers(core[1] + 1, core[1] + 40, 750)
    assert _chi2_pvalue(bad, (0, n), core, *law) < 1e-12


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
        pv = _chi2_pvalue(y, (0, n[k]), _binom_core(n[k], frac),
                          lambda kk: stats.binom.pmf(kk, n[k], frac),
                          lambda kk: stats.binom.cdf(kk, n[k], frac))
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


# ---- the joint law of a channel's placement over its connections -------------
# Sec. III.B: the N_sp walkers a configuration spawns along one part of the
# Liouvillian are distributed over its connected configurations by a
# multinomial law whose cell probabilities are proportional to the elements'
# magnitudes (here with the importance-sampling weights).  The oracle realises
# it as a class split (sequential conditional binomials), a balanced binary tree
# of binomials inside a class, and one categorical pick for a single walker.
# The tests below compare the joint law of the placed counts with the
# multinomial whose cell probabilities come from the connection elements
# (orc.connections, pinned against the Kronecker-form Liouvillian), by chi-square
# over every joint outcome for small counts, and by the means, variances and
# covariances for a large count (a split with the right means but correlated
# cells fails the latter).

def _hop_cells(orc, p, l, m):
    """Cell probabilities of the hop channel over (ket bonds, bra bonds), from the
    connections' imaginary elements."""
    N = p.Lx * p.Ly
    bl = orc.bonds(p.Lx, p.Ly)
    ck, cb, re, im, _, _ = orc.connections(p, l, m)
    el = {(int(a), int(b)): abs(v) for a, b, v in zip(ck, cb, im) if v != 0.0}
    w = []
    for side in (0, 1):
        for s1, s2 in bl:
            mask = (1 << s1) | (1 << s2)
            child = (l ^ mask, m) if side == 0 else (l, m ^ mask)
            w.append(el.get(child, 0.0))
    w = np.array(w)
    assert len(el) == np.count_nonzero(w) and w.sum() > 0
    return w / w.sum(), N


def _joint_chi2(counts, probs, X):
    """Chi-square p-value of sampled count vectors against Multinomial(X, probs)
    over every joint outcome (bins with small expectation pooled)."""
    keep = probs > 0
    assert np.all(counts[:, ~keep] == 0), "a walker placed on a zero-weight cell"
    c = counts[:, keep]
    pk = probs[keep] / probs[keep].sum()
    assert np.all(c.sum(axis=1) == X)
    outcomes, obs = np.unique(c, axis=0, return_counts=True)
    exp = stats.multinomial.pmf(outcomes, X, pk) * len(c)
    # outcomes never seen still carry expectation: the missing mass is one bin
    missing = len(c) - exp.sum()
    order = np.argsort(exp)
    e_b, c_b, e_acc, c_acc = [], [], max(missing, 0.0), 0.0
    for i in order:
        e_acc += exp[i]
        c_acc += obs[i]
        if e_acc >= 20:
            e_b.append(e_acc)
            c_b.append(c_acc)
            e_acc = c_acc = 0.0
    if e_acc > 0:
        e_b[-1] += e_acc
        c_b[-1] += c_acc
    e_b, c_b = np.array(e_b), np.array(c_b)
    return stats.chi2.sf(((c_b - e_b) ** 2 / e_b).sum(), len(e_b) - 1)


def _moments_check(counts, probs, X, zmax=5.0):
    """Means X p, variances X p (1 - p) and covariances -X p_i p_j of the counts."""
    n = len(counts)
    mean = counts.mean(axis=0)
    cov = np.cov(counts.T.astype(float))
    m_exp = X * probs
    c_exp = X * (np.diag(probs) - np.outer(probs, probs))
    # standard error of a sample (co)variance ~ sqrt(var_i var_j / n) for large n
    v = np.maximum(np.diag(c_exp), 1e-300)
    se_mean = np.sqrt(v / n)
    se_cov = np.sqrt(np.outer(v, v) * 2.0 / n)
    live = probs > 0
    zm = np.abs(mean[live] - m_exp[live]) / se_mean[live]
    zc = np.abs(cov - c_exp)[np.ix_(live, live)] / se_cov[np.ix_(live, live)]
    assert zm.max() < zmax, zm.max()
    assert zc.max() < zmax, zc.max()


# (ket, bra) parents on 2x3: an off-diagonal one with a to-diagonal bond (bond
# (0,1) flipped on either side makes it diagonal: the e^{+p} weight), an
# off-diagonal one without, and a diagonal one (all classes e^{-p})
HOP_PARENTS = [(0b000001, 0b000010), (0b000111, 0b000101), (0b010110, 0b010110)]


@pytest.mark.parametrize("l,m", HOP_PARENTS)
@pytest.mark.parametrize("X", [1, 2, 3])
def test_hop_placement_joint_law(orc, l, m, X):
    p = orc.make_params(Lx=2, Ly=3, Jx=0.6, Jy=1.0, Jz=1.2, is_p=0.8, seed=21)
    probs, N = _hop_cells(orc, p, l, m)
    counts = orc.split_many(p, (l << N) | m, 4, X, 120000)
    assert _joint_chi2(counts, probs, X) > PTHRESH


@pytest.mark.parametrize("l,m", HOP_PARENTS[:2])
def test_hop_placement_moments_many_walkers(orc, l, m):
    p = orc.make_params(Lx=2, Ly=3, Jx=0.6, Jy=1.0, Jz=1.2, is_p=0.8, seed=22)
    probs, N = _hop_cells(orc, p, l, m)
    for ch, X in ((4, 37), (8, 400)):
        _moments_check(orc.split_many(p, (l << N) | m, ch, X, 60000), probs, X)


@pytest.mark.parametrize("X", [1, 2, 4, 50])
def test_jump_placement_is_uniform_multinomial(orc, X):
    """The jump channel: every site where ket and bra are both up equally likely."""
    p = orc.make_params(Lx=2, Ly=3, seed=23)
    l, m = 0b110111, 0b011101  # both up on sites 0, 2, 4
    N = 6
    probs = np.zeros(N)
    probs[[0, 2, 4]] = 1.0 / 3.0
    counts = orc.split_many(p, (l << N) | m, 3 if X % 2 else 7, X, 80000)
    if X <= 4:
        assert _joint_chi2(counts, probs, X) > PTHRESH
    else:
        _moments_check(counts, probs, X)


def test_a_split_with_correlated_cells_is_caught(orc):
    """The moment check has teeth: counts with the right means but all walkers
    sent to one cell (perfectly correlated) fail it."""
    rng = np.random.default_rng(3)
    probs = np.array([0.2, 0.3, 0.5])
    X = 20
    cells = rng.choice(3, size=40000, p=probs)
    bad = np.zeros((40000, 3), np.int64)
    bad[np.arange(40000), cells] = X
    with pytest.raises(AssertionError):
        _moments_check(bad, probs, X)
    good = rng.multinomial(X, probs, size=40000)
    _moments_check(good, probs, X)
