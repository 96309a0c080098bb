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



def test_chi_av_closed_forms():
    """chi = c 1 gives |c|; a rank-one chi = u v^T gives |u| |v| 2 / pi (the mean
    of |cos|); a rotation by 90 degrees (the field-across response of a driven
    decaying spin) gives its scale; diag(a, b) gives the ellipse's mean radius."""
    from scipy import integrate
    assert studies.chi_av([[0.7, 0.0], [0.0, 0.7]]) == pytest.approx(0.7, rel=1e-12)
    u, v = np.array([0.3, -0.4]), np.array([1.0, 2.0])
    assert studies.chi_av(np.outer(u, v)) == pytest.approx(
        np.linalg.norm(u) * np.linalg.norm(v) * 2 / np.pi, rel=1e-6)
    assert studies.chi_av([[0.0, -2.0], [2.0, 0.0]]) == pytest.approx(2.0, rel=1e-12)
    a, b = 1.0, 0.25
    ell = integrate.quad(lambda t: np.hypot(a * np.cos(t), b * np.sin(t)), 0, 2 * np.pi)[0]
    assert studies.chi_av([[a, 0.0], [0.0, b]]) == pytest.approx(ell / (2 * np.pi), rel=1e-9)


def test_response_tensor_from_linear_magnetisations():
    """Magnetisations exactly linear in the field give back the tensor."""
    chi = np.array([[0.1, -3.0], [2.6, 0.4]])
    fields = [0.01, 0.02, 0.03]
    m0 = (0.0, 0.0, 1e-4, 1e-4)
    mx = [(chi[0, 0] * h, chi[1, 0] * h, 1e-4, 1e-4) for h in fields]
    my = [(chi[0, 1] * h, chi[1, 1] * h, 1e-4, 1e-4) for h in fields]
    got, se = studies.response_tensor(m0, mx, my, fields)
    assert np.allclose(got, chi, atol=1e-12) and np.all(se > 0)


def test_response_tensor_through_an_exact_zero():
    """A zero-field point with error 0 (exactly 0 by parity) pins the line to
    the origin: the slope is sum w h y / sum w h^2."""
    fields = [0.01, 0.02, 0.03]
    rng = np.random.default_rng(9)
    noise = rng.normal(0, 1e-4, (2, 3, 2))
    m0 = (0.0, 0.0, 0.0, 0.0)
    mx = [(0.5 * h + noise[0, i, 0], -2.0 * h + noise[0, i, 1], 1e-4, 1e-4)
          for i, h in enumerate(fields)]
    my = [(1.5 * h + noise[1, i, 0], 0.2 * h + noise[1, i, 1], 1e-4, 1e-4)
          for i, h in enumerate(fields)]
    chi, se = studies.response_tensor(m0, mx, my, fields)
    h = np.array(fields)
    want = (h * np.array([r[1] for r in mx])).sum() / (h * h).sum()
    assert chi[1, 0] == pytest.approx(want, rel=1e-12)
    assert se[1, 0] == pytest.approx(1e-4 / np.sqrt((h * h).sum()), rel=1e-12)
    assert np.all(np.abs(chi - np.array([[0.5, 1.5], [-2.0, 0.2]])) < 5 * se)
