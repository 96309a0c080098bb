"""The serving loop (continuous batching) with replayed arrivals on a fake
clock: requests are admitted in arrival order, never more projected device
bytes at once than the budget allows, and each served solve's result (its
steps, M_z and SE(M_z), bit for bit) equals the same solve run alone for the
same number of steps."""
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


class FakeClock:
    """Advances a fixed amount every time it is read; sleeping moves it on."""

    def __init__(self, step):
        self.t, self.step = 0.0, step

    def __call__(self):
        self.t += self.step
        return self.t

    def sleep(self, s):
        self.t += s


def _requests(field=False):
    rng = np.random.default_rng(31)
    lat = [(2, 2), (3, 3), (2, 6), (2, 2), (3, 3), (2, 6), (3, 3), (2, 2), (2, 6)]
    reqs = []
    for i, (Lx, Ly) in enumerate(lat):
        t = int(rng.integers(500, 3000))
        reqs.append(dict(arrival=0.1 * i + (0.5 if i >= 6 else 0.0),
                         params=dict(Lx=Lx, Ly=Ly, Jx=float(rng.uniform(0.5, 1.2)), Jy=1.0,
                                     Jz=float(rng.uniform(0.8, 1.2)),
                                     gamma=float(rng.uniform(0.8, 2.0)), dt=0.005, n_a=3,
                                     target_walkers=t, initial_walkers=t, shift_init=0.0,
                                     seed=5, solve_id=200 + i, n_equil=100)))
        if field and i in (2, 5):  # two requests with the in-plane field
            reqs[-1]["params"]["hx"] = 0.1
    return reqs


@pytest.mark.parametrize("budget_solves,graph_k,field", [(2, 0, False), (4, 10, False),
                                                         (4, 10, True)])
def test_replayed_arrivals(dq, budget_solves, graph_k, field):
    """(With field: two of the requests carry the in-plane field, and the pool
    samples every solve by the general routine from the first one on; the
    others alone take the per-entry kernels: the same draws.)"""
    from paper_1802_05931_amd import serving
    reqs = _requests(field)
    max_entries = 30000
    proj = [serving.projected_bytes(r["params"], max_entries) for r in reqs]
    budget = int(budget_solves * max(proj))
    clock = FakeClock(0.02)
    out, st = serving.serve(reqs, slots=8, max_sites=16, hbm_budget=budget, tick=25,
                            se_target=1e-3, min_accum=100, max_steps=300,
                            max_entries=max_entries, graph_k=graph_k, clock=clock,
                            sleep=clock.sleep)
    order = sorted(range(len(reqs)), key=lambda i: reqs[i]["arrival"])
    assert st["admission_order"] == order
    assert st["max_projected_bytes"] <= budget
    assert 1 < st["max_active"] <= budget_solves
    assert st["evicted"] == 0
    for i, r in enumerate(out):
        assert r["admitted"] >= reqs[i]["arrival"]
        assert r["finished"] > r["admitted"]
        assert 0 < r["steps"] <= 300
        _, obs = serving.solve_alone(reqs[i]["params"], r["steps"], tick=25)
        assert obs["step"] == r["steps"]
        for k in ("mz", "se_mz"):
            assert obs[k] == r[k] or (np.isnan(obs[k]) and np.isnan(r[k])), (i, k)
