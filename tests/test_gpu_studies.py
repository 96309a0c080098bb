"""The studies on the device: the initiator extrapolation (Sec. IV.A) on a 2x3
lattice whose exact steady state is known, and the occupancy census
(Sec. IV.B) against the oracle's list sizes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1802_05931_amd as m
    return m


def test_initiator_extrapolation_recovers_the_exact_steady_state(dq):
    """2x3, Jx 0.6, 500 walkers: replicas at n_a = 0, 2, 4, 6, 8 in one batch.
    The thresholds bias M_z (n_a = 8 lies more than 5 standard errors off the
    exact steady state); the straight line through n_a = 2..8 read at n_a -> 0
    lies within 3 of its standard errors of it, as does the n_a = 0 run."""
    from oracle import exact
    from paper_1802_05931_amd import studies
    base = dict(Lx=2, Ly=3, Jx=0.6, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.01, target_walkers=500,
                initial_walkers=500, shift_init=0.0, seed=7, n_equil=2000)
    recs = studies.initiator_runs(base, [0, 2, 4, 6, 8], 60000, graph_k=50)
    ex = exact.observables(exact.ness(2, 3, 0.6, 1.0, 1.0, 1.0), 2, 3)["mz"]
    by = {r["n_a"]: r for r in recs}
    assert all(r["n_accum"] == 58000 for r in recs)
    assert abs(by[0]["mz"] - ex) < 3 * by[0]["se_mz"]
    assert by[8]["mz"] - ex < -5 * by[8]["se_mz"]
    e = studies.extrapolate([r for r in recs if r["n_a"] > 0], "mz")
    print(f"  extrapolated M_z {e['value']:.5f} +- {e['se']:.5f}, exact {ex:.5f}", flush=True)
    assert abs(e["value"] - ex) < 3 * e["se"]
    assert e["slope"] < 0


def test_occupancy_census_equals_the_oracle(dq, orc):
    """A small census (3x3 at 2000 walkers; no initiator, the initiator, and the
    initiator with importance sampling): each run's occupied configurations,
    walkers and diagonal weight are the oracle's after the same steps."""
    from paper_1802_05931_amd import studies
    import workloads
    base = dict(workloads.d2(0.6), target_walkers=2000, initial_walkers=2000, shift_init=0.0)
    rows = studies.occupancy_census(base, [(0, 0.0), (3, 0.0), (3, 1.5)], max_steps=3000,
                                    chunk=500)
    for r in rows:
        o = orc.Oracle(**dict(base, n_a=r["n_a"], is_p=r["is_p"]))
        o.step(r["steps"])
        last = o.last()
        assert (r["entries"], r["walkers"], r["n_w"]) == (last["n_entries"], last["w_tot"],
                                                           last["n_w"]), r
    # the initiator rule and importance sampling each cut the occupied set
    assert rows[1]["entries"] < rows[0]["entries"] and rows[2]["entries"] < rows[1]["entries"]


def test_susceptibility_matches_the_exact_response(dq):
    """The 3 + 3 + 1 field runs of one susceptibility point (Sec. V.B) in one
    batch on 2x2 at n_a = 0: every component of chi_ab = dM_a/dh_b (from lines
    through the runs at h = 0.01, 0.02, 0.03) within 4 standard errors of the
    same lines through the exact steady states, and chi_av likewise.  The
    tensor is far from diagonal (a field along x turns the magnetisation to y)."""
    from oracle import exact
    from paper_1802_05931_amd import studies
    base = dict(Lx=2, Ly=2, Jx=0.9, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.01, n_a=0,
                target_walkers=3000, initial_walkers=3000, shift_init=0.0, seed=17,
                n_equil=3000)
    fields = [0.01, 0.02, 0.03]
    r = studies.susceptibility(base, fields, 60000, graph_k=50)

    def ex(hx, hy):
        o = exact.observables(exact.ness(2, 2, 0.9, 1.0, 1.0, 1.0, hx=hx, hy=hy), 2, 2)
        return (o["mx"], o["my"], 0.0 if hx == hy == 0 else 1e-9, 0.0 if hx == hy == 0 else 1e-9)
    chi_e, _ = studies.response_tensor(ex(0, 0), [ex(h, 0) for h in fields],
                                       [ex(0, h) for h in fields], fields)
    chi, se = np.array(r["chi"]), np.array(r["se_chi"])
    print(f"  chi {chi.tolist()} +- {se.tolist()}; exact {chi_e.tolist()}", flush=True)
    assert np.all(np.abs(chi - chi_e) < 4 * se)
    assert abs(r["chi_av"] - studies.chi_av(chi_e)) < 4 * se.max()
    assert abs(chi_e[1, 0]) > 3.0 and abs(chi_e[0, 0]) < 1e-12
