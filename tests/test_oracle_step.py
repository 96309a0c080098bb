"""Pins of the oracle's whole step against what the paper and the mathematics fix.

* Unbiasedness: the step samples the Euler map of eq. (Euler) for the shifted
  Liouvillian, so E[rho_{n+1} | rho_n] = (1 + dt L~) rho_n exactly (initiator
  off, shift frozen), element by element, with and without importance sampling,
  and also in the regime where a probability exceeds 1 (integer part drawn
  deterministically).
* The initiator rule (Sec. IV.A) removes exactly the progeny of non-initiators on
  unoccupied off-diagonal configurations: the expectation equals the masked map.
* Trace: E[Tr rho_{n+1}] = (1 - dt S) Tr rho_n (trace-preserving L).
* Hermiticity in expectation from a Hermitian start (Sec. III.C: no built-in
  constraint, but the expectation is Hermitian).
* Closed forms: Jx = Jy keeps the list at |dn..dn><dn..dn| bit-exactly and
  gives M_z = -1; the parity selection rule keeps popcount(ket)+popcount(bra) even
  and sigma^x, sigma^y numerators at exactly 0.
* Estimator sums equal Tr(rho O) numerators computed with the Pauli matrices.
* The whole method: the accumulated M_z (and correlators) lie within a few
  standard errors of the exact steady state on 2x2 and 2x3 at n_a = 0.
"""
import numpy as np
import pytest

import workloads
from oracle import exact
from tests.blocking import ratio_se


def _one_step_samples(orc, params, keys, re, im, S, nseed):
    N = params.Lx * params.Ly
    D = 2 ** N
    acc = []
    for seed in range(nseed):
        params.seed = 1000 + seed
        o = orc.Oracle(params)
        o.set_list(keys, re, im)
        o.set_scalars(S, 0, 0, 1)
        o.step(1)
        k, r, i = o.get_list()
        v = np.zeros(D * D, complex)
        v[exact.vec_index(k, N)] = r + 1j * i
        acc.append(v)
        o.close()
    return np.array(acc)


def _z_check(samples, expected, zmax=5.5):
    M = len(samples)
    mean = samples.mean(axis=0)
    for part in (np.real, np.imag):
        sd = part(samples).std(axis=0, ddof=1)
        diff = part(mean) - part(expected)
        fixed = sd == 0
        # no event seen in M samples: the expected change must be small enough
        # for that to be likely (events move at least one walker)
        assert np.all(np.abs(diff[fixed]) < 12.0 / M), "element without events off"
        z = diff[~fixed] / (sd[~fixed] / np.sqrt(M))
        assert np.abs(z).max() < zmax, np.abs(z).max()
        chi = np.mean(z ** 2)
        assert 0.75 < chi < 1.3, chi


CASES = [
    # Lx, Ly, is_p, dt, S, entries, max_pop
    (2, 2, 0.0, 0.01, 0.2, 128, 400),
    (2, 2, 1.5, 0.05, -0.3, 80, 300),
    (2, 3, 0.7, 0.02, 0.1, 250, 200),
    (2, 2, 0.0, 0.6, -1.2, 60, 50),     # probabilities above 1: loud path
]


@pytest.mark.parametrize("Lx,Ly,is_p,dt,S,nent,pop", CASES)
def test_one_step_expectation_is_euler_map(orc, Lx, Ly, is_p, dt, S, nent, pop):
    keys, re, im = workloads.random_list(Lx, Ly, nent, pop, seed=nent + Lx)
    p = orc.make_params(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=dt, n_a=0,
                        is_p=is_p, target_walkers=2 ** 62)
    samples = _one_step_samples(orc, p, keys, re, im, S, nseed=600)
    expected = exact.one_step_expectation(keys, re, im, Lx, Ly, 0.6, 1.0, 1.2, 1.0, dt, S,
                                          is_p=is_p)
    _z_check(samples, expected)
    # trace: E[Tr rho'] = (1 - dt S) Tr rho
    N = Lx * Ly
    D = 2 ** N
    diag = [l * D + l for l in range(D)]
    tr = samples[:, diag].sum(axis=1)
    tr0 = sum(complex(r, i) for k, r, i in zip(keys, re, im)
              if (int(k) >> N) == (int(k) & (D - 1)))
    exp_tr = (1 - dt * S) * tr0
    assert abs(tr.real.mean() - exp_tr.real) < 5.5 * tr.real.std() / np.sqrt(len(tr)) + 1e-9
    assert abs(tr.imag.mean() - exp_tr.imag) < 5.5 * tr.imag.std() / np.sqrt(len(tr)) + 1e-9


def test_initiator_filter_expectation(orc):
    Lx, Ly = 2, 2
    keys, re, im = workloads.random_list(Lx, Ly, 40, 30, seed=5)
    n_a = 20
    p = orc.make_params(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=0.05, n_a=n_a,
                        target_walkers=2 ** 62)
    N = Lx * Ly
    D = 2 ** N
    l = keys >> np.uint64(N)
    m = keys & np.uint64(D - 1)
    non_init = (l != m) & ((np.abs(re.astype(np.int64)) + np.abs(im.astype(np.int64))) <= n_a)
    assert 5 < non_init.sum() < len(keys) - 5
    samples = _one_step_samples(orc, p, keys, re, im, 0.1, nseed=600)
    expected = exact.one_step_expectation(keys, re, im, Lx, Ly, 0.6, 1.0, 1.2, 1.0, 0.05, 0.1,
                                          non_initiator=non_init)
    _z_check(samples, expected)
    # and the unfiltered map is measurably different
    full = exact.one_step_expectation(keys, re, im, Lx, Ly, 0.6, 1.0, 1.2, 1.0, 0.05, 0.1)
    assert np.abs(full - expected).max() > 0.1


def test_hermitian_in_expectation(orc):
    Lx, Ly = 2, 2
    D = 16
    keys, re, im = workloads.random_list(Lx, Ly, 90, 300, seed=9, hermitian=True)
    p = orc.make_params(Lx=Lx, Ly=Ly, dt=0.03, n_a=0, target_walkers=2 ** 62)
    s = _one_step_samples(orc, p, keys, re, im, 0.0, nseed=500)
    mean = s.mean(axis=0).reshape((D, D), order="F")
    sd = s.std(axis=0).reshape((D, D), order="F") / np.sqrt(len(s))
    diff = mean - mean.conj().T
    tol = 6 * np.sqrt(sd ** 2 + sd.T ** 2) + 1e-9
    assert np.all(np.abs(diff.real) <= tol) and np.all(np.abs(diff.imag) <= tol)


def test_xxz_stays_all_down(orc):
    o = orc.Oracle(Lx=3, Ly=3, Jx=0.8, Jy=0.8, dt=0.005, target_walkers=300,
                   initial_walkers=100)
    for _ in range(30):
        o.step(20)
        k, r, i = o.get_list()
        assert k.tolist() == [0] and i.tolist() == [0]
        last = o.last()
        assert last["z"] == -9 * last["t_re"]
    assert o.scalars()["mode"] == 1


def test_parity_rule_and_zero_transverse_numerators(orc):
    o = orc.Oracle(**workloads.D1)
    o.step(3000)
    k, r, i = o.get_list()
    N = 4
    pc = [bin(int(x) >> N).count("1") + bin(int(x) & 15).count("1") for x in k]
    assert all(c % 2 == 0 for c in pc)
    rows = o.series()
    x_col = 3 + orc.SUM_NAMES.index("x")
    y_col = 3 + orc.SUM_NAMES.index("y")
    assert np.all(rows[:, x_col] == 0) and np.all(rows[:, y_col] == 0)


def test_determinism_and_seed_dependence(orc):
    a = orc.Oracle(**dict(workloads.D1, seed=4))
    b = orc.Oracle(**dict(workloads.D1, seed=4))
    c = orc.Oracle(**dict(workloads.D1, seed=5))
    for o in (a, b, c):
        o.step(800)
    ka, ra, ia = a.get_list()
    kb, rb, ib = b.get_list()
    kc, rc, ic = c.get_list()
    assert np.array_equal(ka, kb) and np.array_equal(ra, rb) and np.array_equal(ia, ib)
    assert not (len(ka) == len(kc) and np.array_equal(ka, kc) and np.array_equal(ra, rc))


def test_initiator_threshold_zero_is_no_initiator(orc):
    a = orc.Oracle(**dict(workloads.D1, n_a=0))
    b = orc.Oracle(**dict(workloads.D1, n_a=5, flags=orc.NO_INITIATOR))
    a.step(1500)
    b.step(1500)
    for x, y in zip(a.get_list(), b.get_list()):
        assert np.array_equal(x, y)


def test_estimator_sums_are_trace_numerators(orc):
    Lx, Ly = 2, 3
    N = 6
    D = 64
    keys, re, im = workloads.random_list(Lx, Ly, 400, 50, seed=8)
    o = orc.Oracle(Lx=Lx, Ly=Ly, dt=1e-9, n_a=0, target_walkers=2 ** 62)
    o.set_list(keys, re, im)
    o.set_scalars(0.0, 0, 0, 1)
    o.step(1)                          # dt ~ 0: nothing moves
    k, r, i = o.get_list()
    assert np.array_equal(k, keys) and np.array_equal(r, re) and np.array_equal(i, im)
    s = o.last()
    rho = np.zeros((D, D), complex)
    for kk, rr, ii in zip(k, r, i):
        rho[int(kk) >> N, int(kk) & (D - 1)] = complex(rr, ii)
    tr_num = {}
    for name, op in (("x", exact.SX), ("y", exact.SY), ("z", exact.SZ)):
        tr_num[name] = sum((exact.site_op(op, q, N).multiply(rho.T)).sum().real for q in range(N))
    for name, op in (("cxx", exact.SX), ("cyy", exact.SY), ("czz", exact.SZ)):
        tr_num[name] = sum(((exact.site_op(op, a, N) @ exact.site_op(op, b, N)).multiply(rho.T))
                           .sum().real for a, b in exact.bonds(Lx, Ly))
    for name, v in tr_num.items():
        assert s[name] == round(v), name
    assert s["t_re"] == round(np.trace(rho).real) and s["t_im"] == round(np.trace(rho).imag)
    assert s["n_w"] == int(np.abs(np.diag(rho).real).sum())
    assert s["w_tot"] == int(np.abs(re.astype(np.int64)).sum() + np.abs(im.astype(np.int64)).sum())
    assert s["n_entries"] == len(keys)


@pytest.mark.parametrize("Lx,Ly,steps,target,seed", [(2, 2, 60000, 3000, 1), (2, 3, 20000, 4000, 2)])
def test_ness_within_three_standard_errors(orc, Lx, Ly, steps, target, seed):
    equil = 3000
    o = orc.Oracle(Lx=Lx, Ly=Ly, Jx=0.6, dt=0.01, n_a=0, target_walkers=target,
                   initial_walkers=100, seed=seed, n_equil=equil)
    o.step(steps)
    rows = o.series()
    rows = rows[rows[:, 0] > equil]
    col = {n: 3 + i for i, n in enumerate(orc.SUM_NAMES)}
    rho = exact.ness(Lx, Ly, 0.6, 1.0, 1.0, 1.0)
    ex = exact.observables(rho, Lx, Ly)
    N = Lx * Ly
    nb = len(exact.bonds(Lx, Ly))
    den = rows[:, col["t_re"]]
    mz, se, _ = ratio_se(rows[:, col["z"]] / N, den)
    assert se > 0
    assert abs(mz - ex["mz"]) < 3 * se, (mz, ex["mz"], se)
    for name in ("czz", "cxx", "cyy"):
        v, s2, _ = ratio_se(rows[:, col[name]] / nb, den)
        assert abs(v - ex[name]) < 4 * s2, (name, v, ex[name], s2)
    # the shift fluctuates around the steady-state eigenvalue 0 (Sec. III.A)
    S = rows[:, 1].view(np.float64)
    s_mean, s_se, _ = ratio_se(S, np.ones_like(S))
    assert abs(s_mean) < 4 * s_se + 1e-3


@pytest.mark.parametrize("Lx,Ly,jx,steps,target,seed", [(2, 2, 0.3, 60000, 3000, 3),
                                                        (2, 3, 0.6, 20000, 4000, 4)])
def test_importance_sampled_ness(orc, Lx, Ly, jx, steps, target, seed):
    """Sec. IV.B: with importance sampling (p = 1.5, off-diagonal configurations
    carry weight e^{-p} relative to diagonal ones) the sampled population is the
    weighted density matrix, and the estimators multiply off-diagonal numerators
    by e^{p}.  At n_a = 0 the estimates must still match the exact steady state:
    M_z within 3 standard errors, C_xx, C_yy, C_zz within 4; dividing by the
    weight instead of multiplying would put C_yy e^{-2p} ~ 20x too small, far
    outside.  The oracle's own ratio function (orc.ratios) is checked against
    the same arithmetic done here with numpy."""
    p = 1.5
    equil = 3000
    o = orc.Oracle(Lx=Lx, Ly=Ly, Jx=jx, dt=0.01, n_a=0, is_p=p, target_walkers=target,
                   initial_walkers=100, seed=seed, n_equil=equil)
    o.step(steps)
    rows = o.series()
    rows = rows[rows[:, 0] > equil]
    col = {n: 3 + i for i, n in enumerate(orc.SUM_NAMES)}
    ex = exact.observables(exact.ness(Lx, Ly, jx, 1.0, 1.0, 1.0), Lx, Ly)
    N = Lx * Ly
    nb = len(exact.bonds(Lx, Ly))
    w = np.exp(p)
    den = rows[:, col["t_re"]]
    mz, se, _ = ratio_se(rows[:, col["z"]] / N, den)
    assert abs(mz - ex["mz"]) < 3 * se, (mz, ex["mz"], se)
    got = {}
    for name, f in (("czz", 1.0), ("cxx", w), ("cyy", w)):
        v, s2, _ = ratio_se(rows[:, col[name]] * f / nb, den)
        assert abs(v - ex[name]) < 4 * s2, (name, v, ex[name], s2)
        got[name] = (v, s2)
    # the wrong weight (divided instead of multiplied) is rejected by far
    v, s2 = got["cyy"]
    assert abs(v / w ** 2 - ex["cyy"]) > 10 * s2
    # the oracle's ratios of its accumulated sums: the same numbers
    acc, n_acc = o.acc()
    assert n_acc == len(rows)
    r = orc.ratios(acc, N, nb, p)
    a = dict(zip(orc.SUM_NAMES, acc.tolist()))
    assert r["mz"] == pytest.approx(a["z"] / (N * a["t_re"]), rel=1e-14)
    assert r["cyy"] == pytest.approx(a["cyy"] * w / (nb * a["t_re"]), rel=1e-14)
    assert r["cxx"] == pytest.approx(a["cxx"] * w / (nb * a["t_re"]), rel=1e-14)
    assert r["czz"] == pytest.approx(a["czz"] / (nb * a["t_re"]), rel=1e-14)


def test_shift_update_follows_the_population(orc):
    """Sec. III.C: once the diagonal weight reaches its target, every step sets
    S <- S + (delta / dt) ln(N_w(t) / N_w(t - dt)); before that S stays at its
    start value.  Checked row by row on the step series with numpy's log (the
    oracle uses its own fixed-order log): a factor delta instead of delta / dt,
    a wrong sign or a stale N_w all fail."""
    cfg = dict(workloads.D1, n_equil=0)
    o = orc.Oracle(**cfg)
    o.step(4000)
    rows = o.series()
    S = rows[:, 1].view(np.float64)
    mode = rows[:, 2]
    nw = rows[:, 3 + orc.SUM_NAMES.index("n_w")].astype(np.float64)
    grow = np.where(mode == 0)[0]
    vary = np.where(mode == 1)[0]
    assert len(grow) > 50 and len(vary) > 1000
    assert np.all(S[grow] == cfg["shift_init"])
    # the switch: the first row in vary mode is the first whose N_w reached the target
    first = vary[0]
    assert nw[first] >= cfg["target_walkers"] and np.all(nw[:first] < cfg["target_walkers"])
    assert np.all(np.diff(vary) == 1)  # no return to the growth phase
    k = vary[1:]
    want = S[k - 1] + (cfg["shift_damping"] / cfg["dt"]) * np.log(nw[k] / nw[k - 1])
    assert np.allclose(S[k], want, rtol=0, atol=1e-12)
    assert np.abs(S[k] - S[k - 1]).max() > 1e-3  # the shift does move


@pytest.mark.parametrize("Lx,Ly,is_p,dt,S,nent,pop,hx,hy", [
    (2, 2, 0.0, 0.02, 0.2, 128, 300, 0.3, 0.0),
    (2, 2, 1.5, 0.05, -0.3, 90, 300, 0.1, -0.25),
    (2, 3, 0.7, 0.02, 0.1, 250, 200, -0.2, 0.15),
    (2, 2, 0.0, 0.6, -1.2, 60, 50, 0.4, 0.3),   # probabilities above 1
])
def test_one_step_expectation_with_field(orc, Lx, Ly, is_p, dt, S, nent, pop, hx, hy):
    """Sec. V.B: with the in-plane field the step still samples the Euler map
    (1 + dt L~) rho exactly, now from lists of both parities (the field flips
    one spin), with and without importance sampling."""
    keys, re, im = workloads.random_list(Lx, Ly, nent, pop, seed=nent + Lx + 7, even=False)
    p = orc.make_params(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=dt, n_a=0,
                        is_p=is_p, target_walkers=2 ** 62, hx=hx, hy=hy)
    samples = _one_step_samples(orc, p, keys, re, im, S, nseed=600)
    expected = exact.one_step_expectation(keys, re, im, Lx, Ly, 0.6, 1.0, 1.2, 1.0, dt, S,
                                          is_p=is_p, hx=hx, hy=hy)
    _z_check(samples, expected)


@pytest.mark.parametrize("hx,hy", [(0.15, 0.0), (0.0, 0.15)])
def test_ness_with_field(orc, hx, hy):
    """2x2 at n_a = 0 in a field along x, then along y: the transverse
    magnetisations M_x, M_y (zero without the field) and M_z within 3
    standard errors of the exact steady state in that field."""
    Lx, Ly, jx = 2, 2, 0.6
    equil = 3000
    o = orc.Oracle(Lx=Lx, Ly=Ly, Jx=jx, dt=0.01, n_a=0, target_walkers=3000,
                   initial_walkers=100, seed=11, n_equil=equil, hx=hx, hy=hy)
    o.step(60000)
    rows = o.series()
    rows = rows[rows[:, 0] > equil]
    col = {n: 3 + i for i, n in enumerate(orc.SUM_NAMES)}
    ex = exact.observables(exact.ness(Lx, Ly, jx, 1.0, 1.0, 1.0, hx=hx, hy=hy), Lx, Ly)
    den = rows[:, col["t_re"]]
    for name, key in (("mz", "z"), ("mx", "x"), ("my", "y")):
        v, se, _ = ratio_se(rows[:, col[key]] / 4.0, den)
        assert abs(v - ex[name]) < 3 * se, (name, v, ex[name], se)
    big = "my" if hx else "mx"  # the response is across the field (see test_exact)
    assert abs(ex[big]) > 0.05


@pytest.mark.parametrize("Lx,Ly,is_p,dt,S,nent,pop", [
    (2, 2, 0.0, 0.01, 0.2, 128, 60),
    (2, 2, 1.5, 0.05, -0.3, 80, 60),
    (2, 3, 0.7, 0.02, 0.1, 250, 40),
    (2, 2, 0.0, 0.6, -1.2, 60, 20),     # probabilities above 1
])
def test_per_walker_one_step_expectation(orc, Lx, Ly, is_p, dt, S, nent, pop):
    """The per-walker sampler (Sec. II rules, walker by walker: a uniformly chosen
    connection, spawn probability n_conn dt |element|) samples the same Euler
    map (1 + dt L~) rho as the multinomial one, element by element.  Its
    spawned counts are rarer and larger (one walker's attempt carries the whole
    n_conn-fold probability), so the per-element z-scores are heavier-tailed
    and their mean square needs 2000 samples, not 600, to settle in the
    calibration window."""
    keys, re, im = workloads.random_list(Lx, Ly, nent, pop, seed=nent + Lx + 3)
    p = orc.make_params(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=dt, n_a=0,
                        is_p=is_p, target_walkers=2 ** 62, flags=orc.PER_WALKER)
    samples = _one_step_samples(orc, p, keys, re, im, S, nseed=2000)
    expected = exact.one_step_expectation(keys, re, im, Lx, Ly, 0.6, 1.0, 1.2, 1.0, dt, S,
                                          is_p=is_p)
    _z_check(samples, expected)


def test_per_walker_differs_in_law_but_not_in_mean(orc):
    """Same list, same seeds: the per-walker and the multinomial samplers give
    different lists (different laws for the spawned counts) whose means agree
    with the Euler map (checked above); their death draws are Bsplit in both."""
    keys, re, im = workloads.random_list(2, 2, 60, 30, seed=4)
    a = orc.Oracle(Lx=2, Ly=2, dt=0.05, n_a=0, target_walkers=2 ** 62)
    b = orc.Oracle(Lx=2, Ly=2, dt=0.05, n_a=0, target_walkers=2 ** 62, flags=orc.PER_WALKER)
    for o in (a, b):
        o.set_list(keys, re, im)
        o.set_scalars(0.0, 0, 0, 1)
        o.step(1)
    la, lb = a.get_list(), b.get_list()
    assert not (len(la[0]) == len(lb[0]) and all(np.array_equal(x, y) for x, y in zip(la, lb)))
    with pytest.raises(orc.OracleError):
        orc.Oracle(Lx=2, Ly=2, flags=orc.PER_WALKER, hx=0.1)


def test_per_walker_ness(orc):
    """The per-walker sampler reaches the exact steady state too (2x2, n_a = 0)."""
    Lx, Ly = 2, 2
    equil = 3000
    o = orc.Oracle(Lx=Lx, Ly=Ly, Jx=0.6, dt=0.01, n_a=0, target_walkers=2000,
                   initial_walkers=100, seed=5, n_equil=equil, flags=orc.PER_WALKER)
    o.step(40000)
    rows = o.series()
    rows = rows[rows[:, 0] > equil]
    col = {n: 3 + i for i, n in enumerate(orc.SUM_NAMES)}
    ex = exact.observables(exact.ness(Lx, Ly, 0.6, 1.0, 1.0, 1.0), Lx, Ly)
    mz, se, _ = ratio_se(rows[:, col["z"]] / 4.0, rows[:, col["t_re"]])
    assert abs(mz - ex["mz"]) < 3 * se, (mz, ex["mz"], se)
    v, s2, _ = ratio_se(rows[:, col["cyy"]] / 4.0, rows[:, col["t_re"]])
    assert abs(v - ex["cyy"]) < 4 * s2, (v, ex["cyy"], s2)


def test_per_walker_walker_limit(orc):
    """Walker w of an entry part draws from the stream with draw id
    0x8000 + part 2^13 + (w >> 14), so at most 2^27 walkers fit one part; one
    more fails the step with ORC_ERNG and leaves the list as it was."""
    cfg = dict(workloads.D1, flags=orc.PER_WALKER, target_walkers=2 ** 62)
    o = orc.Oracle(**dict(cfg, initial_walkers=2 ** 27 + 1))
    before = o.get_list()
    with pytest.raises(orc.OracleError) as e:
        o.step(1)
    assert e.value.code == orc.ERNG
    after = o.get_list()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
