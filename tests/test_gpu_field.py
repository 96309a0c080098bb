"""GPU parity with the in-plane field of Sec. V.B (hx sigma^x + hy sigma^y per
site): the quiet scan on the field's probabilities and the general sampling
routine (one thread per entry with events) against the oracle, bit
for bit; and a batch mixing solves with and without the field against each
solve alone (a field-free solve alone takes the quiet scan and the loud and
heavy kernels, in the batch the general path: the same draws)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1802_05931_amd as m
    return m


def _same_list(a, b):
    return (len(a[0]) == len(b[0]) and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            and np.array_equal(a[2], b[2]))


def _run(dq, orc, cfg, chunks, per, graph_k=0):
    g = dq.Solve(dq.make_params(**cfg))
    if graph_k:
        g.set_graph_steps(graph_k)
    o = orc.Oracle(**{k: v for k, v in cfg.items() if k != "capacity_hint"})
    for c in range(chunks):
        g.step(per)
        o.step(per)
        assert _same_list(g.walkers(), o.get_list()), f"list differs after {(c + 1) * per} steps"
        assert g.scalars() == o.scalars()
    assert np.array_equal(g.series(), o.series())
    go = g.observables()
    oacc, n_acc = o.acc()
    assert go["n_accum"] == n_acc and list(go["acc"].values()) == oacc.tolist()
    n = len(g.walkers()[0])
    g.close()
    return go, n


def test_field_2x2(dq, orc):
    cfg = dict(workloads.D1, hx=0.15, n_equil=500)
    go, n = _run(dq, orc, cfg, chunks=6, per=500)
    assert go["acc"]["y"] != 0  # the field along x gives sigma^y
    keys = orc.Oracle(**cfg)
    keys.step(3000)
    k = keys.get_list()[0]
    par = [(bin(int(x) >> 4).count("1") + bin(int(x) & 15).count("1")) % 2 for x in k]
    assert 0 < sum(par) < len(par)  # both parities occupied


@pytest.mark.parametrize("hx,hy,is_p,graph_k", [(0.1, -0.07, 0.0, 0), (0.0, 0.12, 0.5, 10)])
def test_field_3x3(dq, orc, hx, hy, is_p, graph_k):
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=200, hx=hx, hy=hy, is_p=is_p)
    _, n = _run(dq, orc, cfg, chunks=3, per=250, graph_k=graph_k)
    assert n > 2 * 2048


def test_field_5x5_u64(dq, orc):
    cfg = dict(Lx=5, Ly=5, Jx=0.7, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.002, n_a=3, hx=0.05,
               hy=0.03, target_walkers=20000, initial_walkers=20000, shift_init=0.0, n_equil=10,
               seed=3)
    _run(dq, orc, cfg, chunks=2, per=40)


@pytest.mark.parametrize("Lx,Ly,is_p,dt,S,nent,pop,n_a", [
    (2, 2, 0.0, 0.6, -1.2, 100, 50, 0),       # probabilities above 1
    (3, 3, 1.5, 0.02, 0.1, 5000, 300, 3),
    (4, 4, 1.5, 0.002, 0.0, 20000, 40, 3),
])
def test_field_one_step_from_random_lists(dq, orc, Lx, Ly, is_p, dt, S, nent, pop, n_a):
    keys, re, im = workloads.random_list(Lx, Ly, nent, pop, seed=nent + 5, even=False)
    cfg = dict(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=dt, n_a=n_a, is_p=is_p,
               target_walkers=2 ** 62, seed=77, hx=0.21, hy=-0.13)
    g = dq.Solve(dq.make_params(**cfg))
    o = orc.Oracle(**cfg)
    for step in (0, 1, 12345):
        g.set_walkers(keys, re, im)
        g.set_scalars(S, 1, step, 10 ** 6)
        o.set_list(keys, re, im)
        o.set_scalars(S, 1, step, 10 ** 6)
        g.step(1)
        o.step(1)
        assert _same_list(g.walkers(), o.get_list())
        assert g.scalars() == o.scalars()
    g.close()


def test_batch_mixing_field_and_no_field_equals_alone(dq, orc):
    cfgs = [dict(workloads.d2(0.9), solve_id=1, target_walkers=3000, n_equil=100),
            dict(workloads.d2(0.9), solve_id=2, target_walkers=3000, n_equil=100, hx=0.1),
            dict(Lx=2, Ly=6, Jx=0.5, Jz=0.9, gamma=1.3, dt=0.005, n_a=3, target_walkers=2000,
                 initial_walkers=2000, shift_init=0.0, solve_id=3, seed=5, n_equil=50),
            dict(workloads.D1, solve_id=4, n_equil=100, hy=0.2)]
    b = dq.Batch([dq.make_params(**c) for c in cfgs])
    b.set_graph_steps(10)
    alone = []
    for c in cfgs:
        alone.append(dq.Solve(dq.make_params(**c)))
    orcs = [orc.Oracle(**c) for c in cfgs]
    for _ in range(3):
        b.step(200)
        for i, (a, o) in enumerate(zip(alone, orcs)):
            a.step(200)
            o.step(200)
            assert _same_list(b.walkers(i), a.walkers()), i
            assert _same_list(a.walkers(), o.get_list()), i
            assert b.scalars(i) == a.scalars() == o.scalars(), i
    b.close()
    for a in alone:
        a.close()


def test_pool_admits_a_field_solve(dq, orc):
    """A pool switches to the general path when a solve with the field enters;
    the solves before and after keep the oracle's lists."""
    pool = dq.Pool(slots=3, max_sites=16)
    pool.set_graph_steps(10)
    c1 = dict(workloads.d2(1.1), solve_id=21, target_walkers=4000, n_equil=50)
    c2 = dict(workloads.D1, solve_id=22, n_equil=50, hx=0.12, hy=0.05)
    s1 = pool.admit(dq.make_params(**c1))
    pool.step(1)
    o1 = orc.Oracle(**c1)
    pool.step(100)
    o1.step(100)
    s2 = pool.admit(dq.make_params(**c2))
    pool.step(1)
    o1.step(1)
    o2 = orc.Oracle(**c2)
    pool.step(150)
    o1.step(150)
    o2.step(150)
    assert _same_list(pool.walkers(s1), o1.get_list())
    assert _same_list(pool.walkers(s2), o2.get_list())
    assert pool.scalars(s2) == o2.scalars()
    pool.close()


@pytest.mark.parametrize("fork,graph_k", [(1, 0), (-1, 0), (1, 10)],
                         ids=["beside", "after", "beside_in_graphs"])
def test_field_heavy_entries_beside_the_rest(dq, orc, fork, graph_k):
    """Every solve with the field: the entries whose draws are not all small
    go to the scan's heavy list and the general routine, on the second stream
    beside the call-free routine over the rest (fork 1, also inside 10-step
    HIP graphs) or after it (-1); the call-free routine passes on entries with
    20 or more spawns.  A batch of two field solves with large populations
    against the oracle."""
    cfgs = [dict(workloads.D1, solve_id=5, n_equil=100, hx=0.15, target_walkers=20000,
                 initial_walkers=20000),
            dict(workloads.d2(0.6), solve_id=6, target_walkers=50000, initial_walkers=50000,
                 n_equil=100, hy=0.1)]
    b = dq.Batch([dq.make_params(**c) for c in cfgs])
    b.set_heavy_fork(fork)
    if graph_k:
        b.set_graph_steps(graph_k)
    orcs = [orc.Oracle(**c) for c in cfgs]
    for _ in range(3):
        b.step(100)
        for i, o in enumerate(orcs):
            o.step(100)
            assert _same_list(b.walkers(i), o.get_list()), i
            assert b.scalars(i) == o.scalars(), i
    b.close()


@pytest.mark.parametrize("limit", [1, 2, 5])
def test_field_entries_passed_on(dq, orc, limit):
    """The call-free routine passes an entry with `limit` or more walkers
    spawned along one element part by one part of its walkers to the general
    routine (ddqmc_set_field_limit; 20 in production): at 1, every entry with
    a spawn takes that way, at 2 and 5 many.  The oracle's lists either way,
    the passed-on entries counted in the step counts."""
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=100, hx=0.1, hy=-0.07)
    g = dq.Solve(dq.make_params(**cfg))
    g.set_field_limit(limit)
    o = orc.Oracle(**cfg)
    for _ in range(2):
        g.step(200)
        o.step(200)
        assert _same_list(g.walkers(), o.get_list())
        assert g.scalars() == o.scalars()
    assert g.step_counts()[:, 4].sum() > 0
    for bad in (0, 21):
        with pytest.raises(dq.DDQMCError):
            g.set_field_limit(bad)
    g.close()


def test_full_size_field_step(dq, orc):
    """The field workload at full size, as the benchmark times it (the 4x4
    workload with hx 0.05): the GPU steps it to its steady list (about 7.65e7
    entries after some 11,000 steps), where thousands of entries take the
    heavy list on the second stream beside the call-free routine over
    millions of others; then one step from that snapshot against the
    oracle."""
    cfg = dict(workloads.D3, hx=0.05)
    g = dq.Solve(dq.make_params(**cfg))
    g.step(11000)
    keys, re, im = g.walkers()
    sc = g.scalars()
    _, cap = g.device_bytes()
    assert len(keys) > 70_000_000, len(keys)
    assert cap >= 1 << 23  # the fork's threshold (ddqmc_set_heavy_fork mode 0)
    counts = g.step_counts()[-1]
    assert counts[3] > 5_000_000 and counts[4] > 1000  # entries with events, heavy list
    o = orc.Oracle(**cfg)
    o.set_list(keys, re, im)
    o.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
    print(f"  field snapshot at step {sc['step']}: {len(keys)} entries, "
          f"{counts[3]} with events, {counts[4]} heavy", flush=True)
    del keys, re, im
    g.step(1)
    o.step(1)
    assert _same_list(g.walkers(), o.get_list())
    assert g.scalars() == o.scalars()
    print(f"  field step bit-identical ({o.size()} entries)", flush=True)
    g.close()
