"""Host arithmetic of the studies (no GPU): the weighted straight-line fit of
the initiator extrapolation, against numpy's weighted polyfit and the closed
form of a line through exact points; and its error against the spread of
repeated fits of noisy points."""
import numpy as np
import pytest

from paper_1802_05931_amd import studies


def test_line_through_exact_points():
    x = np.array([2.0, 4.0, 8.0, 16.0])
    y = -0.9 + 0.003 * x
    a, sa, b, sb, chi2 = studies.linear_extrapolation(x, y, np.full(4, 1e-3))
    assert a == pytest.approx(-0.9, abs=1e-14) and b == pytest.approx(0.003, abs=1e-15)
    assert chi2 == pytest.approx(0.0, abs=1e-20)


def test_matches_numpy_weighted_polyfit():
    rng = np.random.default_rng(2)
    x = np.array([1.0, 2.0, 3.0, 5.0, 8.0])
    se = rng.uniform(0.5, 2.0, 5) * 1e-3
    y = 0.3 - 0.01 * x + rng.normal(0, 1, 5) * se
    a, sa, b, sb, _ = studies.linear_extrapolation(x, y, se)
    (pb, pa), cov = np.polyfit(x, y, 1, w=1.0 / se, cov="unscaled")
    assert a == pytest.approx(pa, rel=1e-10) and b == pytest.approx(pb, rel=1e-10)
    assert sa == pytest.approx(np.sqrt(cov[1, 1]), rel=1e-10)
    assert sb == pytest.approx(np.sqrt(cov[0, 0]), rel=1e-10)


def test_intercept_error_is_the_spread_of_repeated_fits():
    rng = np.random.default_rng(3)
    x = np.array([2.0, 4.0, 6.0, 8.0])
    se = np.array([1.0, 1.5, 2.0, 3.0]) * 1e-3
    fits = []
    for _ in range(4000):
        y = -0.95 + 0.002 * x + rng.normal(0, 1, 4) * se
        fits.append(studies.linear_extrapolation(x, y, se)[:2])
    fits = np.array(fits)
    assert abs(fits[:, 0].mean() + 0.95) < 4 * fits[0, 1] / np.sqrt(len(fits))
    assert fits[:, 0].std() == pytest.approx(fits[0, 1], rel=0.05)


def test_extrapolate_uses_the_lowest_thresholds():
    recs = [dict(n_a=n, mz=-0.9 + 0.01 * n + (0.5 if n > 10 else 0.0), se_mz=1e-3)
            for n in (1, 2, 4, 8, 25, 75)]
    e = studies.extrapolate(recs, "mz", lowest=4)
    assert e["n_a"] == [1, 2, 4, 8] and e["value"] == pytest.approx(-0.9, abs=1e-12)
    with pytest.raises(ValueError):
        studies.linear_extrapolation([1.0, 1.0], [0.0, 1.0], [1.0, 1.0])
