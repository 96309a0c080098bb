"""GPU parity of walker-by-walker sampling (the rules of Sec. II; flag
PER_WALKER): the prefix / scan / walker kernels against the oracle's
per-walker step, bit for bit, over whole runs and single steps from seeded
random lists (probabilities above 1, entries with more than 2^14 walkers on
one part, 64-bit keys); a batch against each solve alone; and the handles the
mode refuses."""
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
    o = orc.Oracle(**cfg)
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


def test_per_walker_2x2(dq, orc):
    cfg = dict(workloads.D1, n_equil=500, flags=orc.PER_WALKER)
    go, n = _run(dq, orc, cfg, chunks=4, per=500)
    assert go["n_accum"] == 1500 and n > 4


@pytest.mark.parametrize("is_p,n_a,graph_k,per", [(0.0, 3, 0, 250), (0.5, 0, 10, 80)])
def test_per_walker_3x3(dq, orc, is_p, n_a, graph_k, per):
    # (without initiators the list grows fast: fewer steps)
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=200, is_p=is_p, n_a=n_a,
               flags=orc.PER_WALKER)
    _, n = _run(dq, orc, cfg, chunks=3, per=per, graph_k=graph_k)
    assert n > 2 * 2048


def test_per_walker_5x5_u64(dq, orc):
    cfg = dict(Lx=5, Ly=5, Jx=0.7, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.002, n_a=3,
               target_walkers=20000, initial_walkers=20000, shift_init=0.0, n_equil=10, seed=3,
               flags=orc.PER_WALKER)
    _run(dq, orc, cfg, chunks=2, per=40)


@pytest.mark.parametrize("Lx,Ly,is_p,dt,S,nent,pop,n_a", [
    (2, 2, 0.0, 0.6, -1.2, 100, 50, 0),        # probabilities above 1
    (3, 3, 1.5, 0.02, 0.1, 5000, 300, 3),
    (3, 3, 0.5, 0.001, 0.0, 120, 40000, 3),    # more than 2^14 walkers on one part
    (4, 4, 1.5, 0.002, 0.0, 20000, 40, 3),
])
def test_per_walker_one_step_from_random_lists(dq, orc, Lx, Ly, is_p, dt, S, nent, pop, n_a):
    keys, re, im = workloads.random_list(Lx, Ly, nent, pop, seed=nent + 9)
    cfg = dict(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=dt, n_a=n_a, is_p=is_p,
               target_walkers=2 ** 62, seed=78, flags=orc.PER_WALKER)
    g = dq.Solve(dq.make_params(**cfg))
    o = orc.Oracle(**cfg)
    for step in (0, 1, 12345):
        g.set_walkers(keys, re, im)
        g.set_scalars(S, 1, step, 10 ** 6)
        o.set_list(keys, re, im)
        o.set_scalars(S, 1, step, 10 ** 6)
        g.step(1)
        o.step(1)
        assert _same_list(g.walkers(), o.get_list()), step
        assert g.scalars() == o.scalars()
    g.close()


def test_per_walker_batch_equals_alone(dq, orc):
    cfgs = [dict(workloads.d2(0.9), solve_id=1, target_walkers=3000, n_equil=100),
            dict(Lx=2, Ly=6, Jx=0.5, Jz=0.9, gamma=1.3, dt=0.005, n_a=3, target_walkers=2000,
                 initial_walkers=2000, shift_init=0.0, solve_id=3, seed=5, n_equil=50),
            dict(workloads.D1, solve_id=4, n_equil=100)]
    cfgs = [dict(c, flags=orc.PER_WALKER) for c in cfgs]
    b = dq.Batch([dq.make_params(**c) for c in cfgs])
    b.set_graph_steps(10)
    orcs = [orc.Oracle(**c) for c in cfgs]
    for _ in range(3):
        b.step(200)
        for i, o in enumerate(orcs):
            o.step(200)
            assert _same_list(b.walkers(i), o.get_list()), i
            assert b.scalars(i) == o.scalars(), i
    b.close()


def test_per_walker_refusals(dq, orc):
    pw = dict(workloads.D1, flags=orc.PER_WALKER)
    with pytest.raises(dq.DDQMCError):
        dq.Solve(dq.make_params(**dict(pw, hx=0.1)))
    with pytest.raises(dq.DDQMCError):
        dq.Batch([dq.make_params(**pw), dq.make_params(**dict(workloads.D1, solve_id=1))])
    pool = dq.Pool(slots=2, max_sites=9)
    with pytest.raises(dq.DDQMCError):
        pool.admit(dq.make_params(**pw))
    pool.close()


def test_per_walker_walker_limit(dq, orc):
    """More than 2^27 walkers on one part of one entry: the step fails with
    DDQMC_ERNG (as the oracle's with ORC_ERNG) and the list and scalars stay
    at the last completed step."""
    cfg = dict(workloads.D1, flags=orc.PER_WALKER, target_walkers=2 ** 62,
               initial_walkers=2 ** 27 + 1)
    g = dq.Solve(dq.make_params(**cfg))
    before, sc = g.walkers(), g.scalars()
    with pytest.raises(dq.DDQMCError) as e:
        g.step(1)
    assert e.value.code == -8
    assert _same_list(before, g.walkers()) and g.scalars() == sc
    o = orc.Oracle(**cfg)
    with pytest.raises(orc.OracleError) as eo:
        o.step(1)
    assert eo.value.code == orc.ERNG
    g.close()
