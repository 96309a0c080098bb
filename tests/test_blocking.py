"""The standard errors of the ratio estimators (the paper gives no error
analysis; here Flyvbjerg-Petersen blocking of the per-step series with the
delta method for the ratio of means).

The test helper tests/blocking.ratio_se is pinned against series whose error
of the mean is known in closed form: independent normals (sigma / sqrt(n)) and
an AR(1) process x_t = phi x_{t-1} + e_t, whose mean over n steps has variance
sigma_x^2 (1 + phi) / ((1 - phi) n) for large n; and a ratio with a constant
denominator reduces to the numerator's error divided by it.  The library's own
routine (ddqmc_ratio_se, used by ddqmc_observables and by the serving stop
rule) must return the helper's value on the same series."""
import numpy as np
import pytest

from tests.blocking import ratio_se


@pytest.fixture(scope="module")
def dq():
    import os
    from paper_1802_05931_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    import paper_1802_05931_amd as m
    return m


def _ar1(n, phi, rng, sigma_e=1.0):
    e = rng.normal(0.0, sigma_e, n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


def test_independent_series(dq):
    rng = np.random.default_rng(1)
    n = 1 << 16
    x = rng.normal(3.0, 2.0, n)
    m, se, _ = ratio_se(x, np.ones(n))
    assert abs(m - x.mean()) < 1e-12
    assert abs(se / (2.0 / np.sqrt(n)) - 1.0) < 0.12


@pytest.mark.parametrize("phi", [0.5, 0.9, 0.97])
def test_ar1_error_of_the_mean(dq, phi):
    rng = np.random.default_rng(int(phi * 100))
    n = 1 << 17
    x = 5.0 + _ar1(n, phi, rng)
    sigma_x2 = 1.0 / (1 - phi * phi)
    want = np.sqrt(sigma_x2 * (1 + phi) / ((1 - phi) * n))
    _, se, _ = ratio_se(x, np.ones(n))
    # the plateau of the blocking curve; the naive error is sqrt((1+phi)/(1-phi)) smaller
    assert abs(se / want - 1.0) < 0.2, (se, want)
    naive = x.std() / np.sqrt(n)
    assert se > 1.5 * naive


def test_ratio_with_a_constant_denominator(dq):
    rng = np.random.default_rng(7)
    n = 1 << 14
    x = 1.0 + _ar1(n, 0.8, rng)
    _, se1, _ = ratio_se(x, np.ones(n))
    _, se4, _ = ratio_se(x, 4.0 * np.ones(n))
    assert abs(se4 - se1 / 4.0) < 1e-12


@pytest.mark.parametrize("n,phi,seed", [(16, 0.0, 1), (1000, 0.7, 2), (50000, 0.95, 3),
                                        (70001, 0.6, 4), (15, 0.5, 5)])
def test_library_error_equals_the_helper(dq, n, phi, seed):
    rng = np.random.default_rng(seed)
    den = 1000.0 + 30.0 * _ar1(n, phi, rng)
    num = -0.9 * den + 5.0 * _ar1(n, phi, rng)
    got = dq.ratio_se(num, den)
    want = ratio_se(num, den)[1] if n >= 16 else 0.0
    assert got == pytest.approx(want, rel=1e-10, abs=1e-300)
