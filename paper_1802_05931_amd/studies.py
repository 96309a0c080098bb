"""Studies built on the step: the initiator extrapolation (Sec. IV.A) and the
census of occupied density-matrix elements (Sec. IV.B), both run through the
library's handles (every step in its kernels); this module only arranges the
runs and reduces their observables.

Initiator extrapolation (Sec. IV.A, last paragraph, and the initiator figure):
the initiator rule biases the estimates; runs at decreasing thresholds I_limit
(n_a) are fitted with a straight line through the lowest thresholds, and the
line's value at I_limit -> 0 is the estimate.  The runs are replicas of one
batch (one launch per stage for all thresholds), each with its own n_a and
solve id.

Occupancy census (Sec. IV.B, the occupied-element figure): how many
configurations the walker list occupies at a given population, with and
without the initiator rule and importance sampling.

Susceptibility (Sec. V.B): the linear response of the transverse
magnetisation to the in-plane field, chi_ab = dM_a / dh_b at h = 0, from 3 + 3
+ 1 runs (three field strengths along x, three along y, one without field) in
one batch, and the angle-averaged chi_av = (1 / 2 pi) int |chi (cos t, sin t)| dt.
"""
import numpy as np

from . import Batch, Solve, make_params
from ._lib import ECAPACITY, DDQMCError

OBS = ("mz", "mx", "my", "cxx", "cyy", "czz")


def linear_extrapolation(x, y, se):
    """Weighted least-squares line y = a + b x through points with standard
    errors se; returns (a, se(a), b, se(b), chi2 per degree of freedom).  The
    line's value at x = 0 is the extrapolated estimate."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    w = 1.0 / np.asarray(se, float) ** 2
    S, Sx, Sy = w.sum(), (w * x).sum(), (w * y).sum()
    Sxx, Sxy = (w * x * x).sum(), (w * x * y).sum()
    det = S * Sxx - Sx * Sx
    if not det > 0:
        raise ValueError("linear_extrapolation: need two distinct x with finite errors")
    a = (Sxx * Sy - Sx * Sxy) / det
    b = (S * Sxy - Sx * Sy) / det
    dof = len(x) - 2
    chi2 = float((w * (y - a - b * x) ** 2).sum() / dof) if dof > 0 else float("nan")
    return a, np.sqrt(Sxx / det), b, np.sqrt(S / det), chi2


def initiator_runs(base, n_a_values, steps, graph_k=0, stream=None, tile_rows=None, chunk=0,
                   log=None):
    """Replicas of one solve at the given initiator thresholds, stepped together
    in one batch for ``steps`` steps (in chunks of ``chunk`` steps with a log
    line each, if given).  Returns one record per threshold: n_a and the
    accumulated ratios with their standard errors."""
    cfgs = [dict(base, n_a=int(n), solve_id=int(base.get("solve_id", 0)) + i)
            for i, n in enumerate(n_a_values)]
    b = Batch([make_params(**c) for c in cfgs], stream=stream)
    if graph_k:
        b.set_graph_steps(graph_k)
    if tile_rows:
        b.set_tile_table([tuple(r) for r in tile_rows])
    done = 0
    while done < steps:
        n = min(chunk or steps, steps - done)
        b.step(n)
        done += n
        if log:
            log(f"initiator runs: {done} of {steps} steps, {b.list_size()} entries")
    out = []
    for i, n in enumerate(n_a_values):
        o = b.observables(i)
        rec = dict(n_a=int(n), n_accum=int(o["n_accum"]), entries=int(o["last"]["n_entries"]))
        for k in OBS:
            rec[k] = float(o[k])
            rec["se_" + k] = float(o["se_" + k])
        out.append(rec)
    b.close()
    return out


def extrapolate(records, obs="mz", lowest=None):
    """The initiator extrapolation of one observable: a line through the records
    with the `lowest` smallest thresholds (all by default), read at n_a = 0."""
    rs = sorted(records, key=lambda r: r["n_a"])
    if lowest:
        rs = rs[:lowest]
    a, sa, b, sb, chi2 = linear_extrapolation([r["n_a"] for r in rs], [r[obs] for r in rs],
                                              [r["se_" + obs] for r in rs])
    return dict(obs=obs, value=a, se=sa, slope=b, se_slope=sb, chi2_dof=chi2,
                n_a=[r["n_a"] for r in rs])


def occupancy_census(base, grid, max_steps, chunk=500, tol=0.01, cap_limit=0, stream=None,
                     log=None):
    """For each (n_a, is_p) of `grid`: a solve of `base` stepped in chunks until
    its list changes by less than `tol` over two chunks (or max_steps), then its
    occupied configurations, walkers and diagonal weight.  A run whose list
    outgrows cap_limit entries (0: no limit) is reported with exceeded=True."""
    rows = []
    for n_a, p in grid:
        cfg = dict(base, n_a=int(n_a), is_p=float(p))
        g = Solve(make_params(**cfg), stream=stream)
        if cap_limit:
            g.set_capacity_limit(int(cap_limit))
        sizes, done, exceeded = [], 0, False
        try:
            while done < max_steps:
                g.step(chunk)
                done += chunk
                sizes.append(g.list_size())
                if len(sizes) >= 3 and abs(sizes[-1] - sizes[-3]) <= tol * sizes[-1]:
                    break
        except DDQMCError as e:
            if e.code != ECAPACITY:
                raise
            exceeded = True
        last = g.observables()["last"]
        row = dict(n_a=int(n_a), is_p=float(p), steps=int(g.scalars()["step"]),
                   steady=bool(len(sizes) >= 3 and not exceeded and
                               abs(sizes[-1] - sizes[-3]) <= tol * sizes[-1]),
                   exceeded=exceeded, entries=int(last["n_entries"]),
                   walkers=int(last["w_tot"]), n_w=int(last["n_w"]),
                   entries_per_walker=float(last["n_entries"]) / max(int(last["w_tot"]), 1))
        rows.append(row)
        if log:
            log(f"census n_a {n_a} p {p}: {row}")
        g.close()
    return rows


def chi_av(chi, n=3600):
    """Angle average (1 / 2 pi) int_0^{2 pi} |chi (cos t, sin t)^T| dt of a 2x2
    response tensor, by the midpoint rule over n angles (the integrand is
    periodic, so the rule converges fast)."""
    chi = np.asarray(chi, float)
    t = (np.arange(n) + 0.5) * (2.0 * np.pi / n)
    v = chi @ np.vstack([np.cos(t), np.sin(t)])
    return float(np.mean(np.hypot(v[0], v[1])))


def response_tensor(m0, mx_runs, my_runs, fields):
    """chi_ab from magnetisations: m0 = (M_x, M_y, se_x, se_y) without field;
    mx_runs / my_runs the same with the field along x / y at the strengths
    `fields`.  chi_ab is the slope of a weighted line through M_a at h_b = 0
    and the three fields along b (through the zero-field point itself when its
    error is 0, as it is exactly 0 by the parity rule); returns (chi, se(chi))."""
    chi = np.zeros((2, 2))
    se = np.zeros((2, 2))
    h = np.concatenate([[0.0], np.asarray(fields, float)])
    for b, runs in enumerate((mx_runs, my_runs)):
        for a in range(2):
            y = np.array([m0[a]] + [r[a] for r in runs])
            e = np.array([m0[2 + a]] + [r[2 + a] for r in runs])
            if e[0] == 0.0:
                # without the field the transverse magnetisation is exactly 0 (the
                # parity rule): the line goes through that point
                w = 1.0 / e[1:] ** 2
                hh = h[1:]
                chi[a, b] = float((w * hh * (y[1:] - y[0])).sum() / (w * hh * hh).sum())
                se[a, b] = float(1.0 / np.sqrt((w * hh * hh).sum()))
            else:
                _, _, slope, s_slope, _ = linear_extrapolation(h, y, e)
                chi[a, b] = slope
                se[a, b] = s_slope
    return chi, se


def susceptibility(base, fields, steps, graph_k=0, stream=None, chunk=0, log=None):
    """The 3 + 3 + 1 runs of one susceptibility point in one batch: no field,
    the field along x at each strength of `fields`, then along y.  Returns chi,
    its standard errors, chi_av and the runs' magnetisations."""
    cfgs = [dict(base, hx=0.0, hy=0.0)]
    cfgs += [dict(base, hx=float(h), hy=0.0) for h in fields]
    cfgs += [dict(base, hx=0.0, hy=float(h)) for h in fields]
    for i, c in enumerate(cfgs):
        c["solve_id"] = int(base.get("solve_id", 0)) + i
    b = Batch([make_params(**c) for c in cfgs], stream=stream)
    if graph_k:
        b.set_graph_steps(graph_k)
    done = 0
    while done < steps:
        k = min(chunk or steps, steps - done)
        b.step(k)
        done += k
        if log:
            log(f"susceptibility runs: {done} of {steps} steps, {b.list_size()} entries")
    m = []
    for i in range(len(cfgs)):
        o = b.observables(i)
        m.append((o["mx"], o["my"], o["se_mx"], o["se_my"]))
    b.close()
    nf = len(fields)
    chi, se = response_tensor(m[0], m[1:1 + nf], m[1 + nf:], fields)
    return dict(chi=chi.tolist(), se_chi=se.tolist(), chi_av=chi_av(chi), runs=m,
                fields=[float(h) for h in fields])
