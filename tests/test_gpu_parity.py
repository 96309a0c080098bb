"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Walker lists, shifts and integer estimator sums must be bit-identical to the
oracle on the same Philox streams (integer work: bit-exact; the fp64 sampling
arithmetic has a fixed operation order on both sides, so it is bit-exact too).
Cases span several sort and merge tiles with ragged tails, u32 and u64 keys,
importance sampling, the initiator filter, buffer regrowth, batched and served
solves, the error paths, and a window of the full-size 4x4 workload.
"""
import os
import time

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


def _compare_run(dq, orc, cfg, chunks, per, check_series=True, fork=0, tree_queue=0,
                 stats=None, loud_grid=0):
    g = dq.Solve(dq.make_params(**cfg))
    g.set_heavy_fork(fork)
    g.set_tree_queue(tree_queue)
    g.set_loud_grid(loud_grid)
    o = orc.Oracle(**{k: v for k, v in cfg.items() if k != "capacity_hint"})
    for c in range(chunks):
        g.step(per)
        o.step(per)
        gl = g.walkers()
        ol = o.get_list()
        assert _same_list(gl, ol), f"list differs after {(c + 1) * per} steps"
        print(f"  {cfg['Lx']}x{cfg['Ly']}: {(c + 1) * per} steps, {len(gl[0])} entries ok",
              flush=True)
        gs, os_ = g.scalars(), o.scalars()
        assert gs == os_, (gs, os_)
    if check_series:
        assert np.array_equal(g.series(), o.series())
    go = g.observables()
    oacc, n_acc = o.acc()
    assert go["n_accum"] == n_acc
    assert list(go["acc"].values()) == oacc.tolist()
    ratios = orc.ratios(oacc, o.N, len(orc.bonds(cfg["Lx"], cfg["Ly"])), cfg.get("is_p", 0.0))
    for k, v in ratios.items():
        assert go[k] == v or (np.isnan(go[k]) and np.isnan(v)), k
    n = len(gl[0])
    if stats is not None:
        stats["general_path_entries"] = int(g.step_counts()[:, 4].sum())
    g.close()
    return n


def test_device_math_bit_exact(dq, orc):
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(0, 1, 4000), np.exp(rng.uniform(-700, 700, 4000)),
                        rng.uniform(0.5, 2, 2000), [1.0, 2.0, 5e-324, 1e-310, 0.75]])
    out = dq.dev_math(x)
    assert np.array_equal(out[:, 0], np.array([orc.det_log(v) for v in x]))
    xe = rng.uniform(-700, 700, 3000)
    oute = dq.dev_math(xe)
    assert np.array_equal(oute[:, 1], np.array([orc.det_exp(v) for v in xe]))
    assert np.array_equal(out[:, 2], np.sqrt(x)), "device sqrt is not correctly rounded"
    with np.errstate(over="ignore"):  # 1 / 5e-324 overflows to inf on both sides
        recip = 1.0 / x
    assert np.array_equal(out[:, 3], recip), "device division is not correctly rounded"


def test_device_quiet_test_matches_the_product(dq, orc):
    """The scan's quiet test (a single-precision estimate of the no-event
    probability with an error band, the fp64 product inside the band) must
    decide u < g exactly as the oracle's product g does, also for uniforms
    placed on both sides of g at the band's edges and one ulp away."""
    rng = np.random.default_rng(12)
    m = 1500
    p = rng.uniform(0, 0.06, (m, 4)) * (rng.random((m, 4)) < 0.85)
    p[: m // 10] = rng.uniform(0, 0.9, (m // 10, 4))        # p > 1/2: the product path
    n = rng.integers(0, 40, (m, 2))
    n[m // 10: m // 5] = rng.integers(0, 3000, (m // 10, 2))  # n > 1024: the product path
    n[n.sum(axis=1) == 0, 0] = 1
    g = np.array([orc.no_event_prob(np.tile(p[i], 2), np.repeat(n[i], 4)) for i in range(m)])
    mg = 1e-5 * (1.0 + n.sum(axis=1))
    rel = [0.0, -1e-12, 1e-12, -1e-7, 1e-7, -0.5, 0.5, -1.0, 1.0, -1.01, 1.01, -2.0, 2.0]
    us, ps, ns, gs = [], [], [], []
    for r in rel:
        us.append(g * (1.0 + r * mg) if r not in (0.0,) else g.copy())
        ps.append(p)
        ns.append(n)
        gs.append(g)
    for d in (-np.inf, np.inf):  # one ulp below and above
        us.append(np.nextafter(g, d))
        ps.append(p)
        ns.append(n)
        gs.append(g)
    us.append(rng.random(m))
    ps.append(p)
    ns.append(n)
    gs.append(g)
    u, pa, na, ga = (np.concatenate(x) for x in (us, ps, ns, gs))
    keep = (u >= 0) & (u < 1)
    u, pa, na, ga = u[keep], pa[keep], na[keep], ga[keep]
    out = dq.dev_quiet(pa, na, u)
    assert np.array_equal(out & 1, (u < ga).astype(np.int32))
    est = (out & 2) != 0
    assert est.sum() > len(u) // 6 and (~est).sum() > len(u) // 6  # both paths taken
    with pytest.raises(dq.DDQMCError):
        dq.dev_quiet([[1.0, 0, 0, 0]], [[1, 0]], [0.5])


def test_device_uniforms_bit_exact(dq, orc):
    for args in [(0, 0, 0, 0, 0), (0x123456789ABCDEF0, 17, 0xDEADBEEF12, 44, 3077),
                 (2 ** 64 - 1, 65535, 2 ** 64 - 1, 2 ** 32 - 1, 0xFFFF)]:
        assert np.array_equal(dq.dev_uniforms(*args, 5000), orc.uniforms(*args, 5000))


@pytest.mark.parametrize("n,p,mode", [(1, 0.3, 0), (7, 0.2, 0), (200, 0.049, 0), (1000, 0.3, 0),
                                      (100000, 0.02, 0), (2 ** 31 - 1, 1e-6, 0), (300, 0.9, 0),
                                      (30, 0.34, 0), (5, 0.01, 1), (400, 0.1, 1), (5, 0.8, 1),
                                      (20000, 0.001, 1), (3, 2.4, 2), (1000, 3.05, 2)])
def test_device_binomials_bit_exact(dq, orc, n, p, mode):
    assert np.array_equal(dq.dev_binom(n, p, mode, 11, 20000), orc.binom_many(n, p, mode, 11, 20000))


def test_plain_2x2_d1(dq, orc):
    cfg = dict(workloads.D1)
    n = _compare_run(dq, orc, cfg, chunks=10, per=300)
    assert n > 5


@pytest.mark.parametrize("fork,loud_grid", [(0, 0), (1, 0), (0, 1), (1, 2)])
def test_plain_3x3_jx06(dq, orc, fork, loud_grid):
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=200)
    n = _compare_run(dq, orc, cfg, chunks=4, per=250, fork=fork, loud_grid=loud_grid)
    assert n > 2 * 2048, "should span several tiles"


def test_plain_2x6_initiator_off(dq, orc):
    cfg = dict(Lx=2, Ly=6, Jx=0.5, Jy=1.0, Jz=0.8, gamma=0.7, dt=0.005, n_a=0,
               target_walkers=3000, initial_walkers=3000, shift_init=0.0, n_equil=50, seed=9)
    _compare_run(dq, orc, cfg, chunks=3, per=60)


@pytest.mark.parametrize("fork", [0, 1])
def test_5x5_u64_keys(dq, orc, fork):
    cfg = dict(Lx=5, Ly=5, Jx=0.7, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.002, n_a=3,
               target_walkers=20000, initial_walkers=20000, shift_init=0.0, n_equil=10, seed=3)
    _compare_run(dq, orc, cfg, chunks=3, per=40, fork=fork)


@pytest.mark.parametrize("lattice,places", [("3x3", 1), ("3x3", 6), ("5x5", 2)])
def test_tree_queue_full_takes_the_general_path(dq, orc, lattice, places):
    """With a member-tree queue of a few places most entries with trees find no
    room and take the general path: the lists stay the oracle's, and more
    entries take the general path than with the full queue."""
    if lattice == "3x3":
        cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=200)
        chunks, per = 2, 250
    else:
        cfg = dict(Lx=5, Ly=5, Jx=0.7, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.002, n_a=3,
                   target_walkers=20000, initial_walkers=20000, shift_init=0.0, n_equil=10,
                   seed=3)
        chunks, per = 2, 40
    full, small = {}, {}
    _compare_run(dq, orc, cfg, chunks=chunks, per=per, stats=full)
    _compare_run(dq, orc, cfg, chunks=chunks, per=per, tree_queue=places, stats=small)
    assert small["general_path_entries"] > full["general_path_entries"], (small, full)


@pytest.mark.parametrize("Lx,Ly,is_p,dt,S,nent,pop,n_a", [
    (2, 2, 0.0, 0.6, -1.2, 100, 50, 0),        # probabilities above 1
    (3, 3, 1.5, 0.02, 0.1, 5000, 300, 3),     # IS + filter, many tiles
    (4, 4, 1.5, 0.002, 0.0, 20000, 40, 3),    # the 4x4 workload's parameters
    (2, 6, 0.7, 0.01, 0.3, 9000, 1000, 50),
])
def test_one_step_from_random_lists(dq, orc, Lx, Ly, is_p, dt, S, nent, pop, n_a):
    keys, re, im = workloads.random_list(Lx, Ly, nent, pop, seed=nent)
    cfg = dict(Lx=Lx, Ly=Ly, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=dt, n_a=n_a, is_p=is_p,
               target_walkers=2 ** 62, seed=77)
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


def test_regrow_tiny_capacity(dq, orc):
    cfg = dict(workloads.d2(0.6), target_walkers=20000, capacity_hint=16, n_equil=100)
    _compare_run(dq, orc, cfg, chunks=2, per=300)


def test_batch_equals_alone(dq, orc):
    cfgs = [dict(workloads.D1, solve_id=0, n_equil=100),
            dict(workloads.d2(0.9), solve_id=1, target_walkers=3000, n_equil=100),
            dict(Lx=2, Ly=6, Jx=0.5, Jz=0.9, gamma=1.3, dt=0.005, n_a=3, target_walkers=2000,
                 initial_walkers=2000, shift_init=0.0, solve_id=2, seed=5, n_equil=50),
            dict(workloads.D1, solve_id=3, seed=8, n_equil=100)]
    b = dq.Batch([dq.make_params(**c) for c in cfgs])
    orcs = [orc.Oracle(**c) for c in cfgs]
    for _ in range(3):
        b.step(200)
        for i, o in enumerate(orcs):
            o.step(200)
            assert _same_list(b.walkers(i), o.get_list()), i
            assert b.scalars(i) == o.scalars(), i
    for i, o in enumerate(orcs):
        assert np.array_equal(b.series(i), o.series())
    b.close()


def test_pool_admit_retire_equals_alone(dq, orc):
    pool = dq.Pool(slots=4, max_sites=16)
    c1 = dict(workloads.d2(1.1), solve_id=11, target_walkers=4000, n_equil=50)
    c2 = dict(Lx=4, Ly=4, Jx=0.8, Jy=1.0, Jz=1.0, gamma=1.5, dt=0.005, n_a=3, is_p=0.0,
              target_walkers=5000, initial_walkers=5000, shift_init=0.0, solve_id=12, n_equil=50)
    c3 = dict(workloads.D1, solve_id=13, n_equil=50)
    s1 = pool.admit(dq.make_params(**c1))
    pool.step(1)                 # s1 enters the list
    o1 = orc.Oracle(**c1)
    pool.step(150)
    o1.step(150)
    s2 = pool.admit(dq.make_params(**c2))
    pool.step(1)
    o1.step(1)
    o2 = orc.Oracle(**c2)
    pool.step(100)
    o1.step(100)
    o2.step(100)
    assert _same_list(pool.walkers(s1), o1.get_list())
    assert _same_list(pool.walkers(s2), o2.get_list())
    pool.retire(s1)
    s3 = pool.admit(dq.make_params(**c3))
    assert s3 != s1
    pool.step(1)
    o2.step(1)
    o3 = orc.Oracle(**c3)
    assert len(pool.walkers(s1)[0]) == 0
    pool.step(120)
    o2.step(120)
    o3.step(120)
    assert _same_list(pool.walkers(s2), o2.get_list())
    assert _same_list(pool.walkers(s3), o3.get_list())
    assert np.array_equal(pool.series(s3), o3.series())
    assert pool.scalars(s2) == o2.scalars()
    pool.close()


@pytest.mark.parametrize("fork", [0, 1])
def test_graph_steps_equal_eager(dq, orc, fork):
    """k-step HIP graphs (replayed several times per call, re-captured after
    the buffers grow from a tiny capacity and after the tree queue shrinks)
    give the eager launches' lists, which the oracle checks too; with fork = 1
    the heavy entries run on the second stream (fork and join inside the
    graph)."""
    cfg = dict(workloads.d2(0.6), target_walkers=20000, capacity_hint=16, n_equil=60)
    a = dq.Solve(dq.make_params(**cfg))
    b = dq.Solve(dq.make_params(**cfg))
    b.set_heavy_fork(fork)
    b.set_graph_steps(10)
    o = orc.Oracle(**{k: v for k, v in cfg.items() if k != "capacity_hint"})
    for i, per in enumerate((35, 35, 120, 7, 64)):
        if i == 2:
            b.set_loud_grid(1)  # another loud grid: the graph is captured again
        if i == 3:
            b.set_tree_queue(2)  # a new kernel argument: the graph is captured again
        a.step(per)
        b.step(per)
        o.step(per)
        assert _same_list(a.walkers(), b.walkers())
        assert _same_list(b.walkers(), o.get_list())
        assert a.scalars() == b.scalars() == o.scalars()
        print(f"  graph steps: {o.scalars()['step']} steps, {len(o.get_list()[0])} entries ok",
              flush=True)
    assert np.array_equal(b.series(), o.series())
    b.set_graph_steps(0)
    a.step(20)
    b.step(20)
    assert _same_list(a.walkers(), b.walkers())
    a.close()
    b.close()


@pytest.mark.parametrize("fork", [0, 1])
def test_graph_steps_batch_equals_alone(dq, orc, fork):
    cfgs = [dict(workloads.D1, solve_id=0, n_equil=40),
            dict(workloads.d2(0.9), solve_id=1, target_walkers=3000, n_equil=40),
            dict(workloads.D1, solve_id=2, seed=3, n_equil=40)]
    b = dq.Batch([dq.make_params(**c) for c in cfgs])
    b.set_heavy_fork(fork)
    b.set_graph_steps(16)
    orcs = [orc.Oracle(**c) for c in cfgs]
    for per in (48, 100):
        b.step(per)
        for i, o in enumerate(orcs):
            o.step(per)
            assert _same_list(b.walkers(i), o.get_list()), i
            assert b.scalars(i) == o.scalars(), i
    b.close()


def test_graph_steps_invalid(dq):
    from paper_1802_05931_amd import DDQMCError
    g = dq.Solve(dq.make_params(**workloads.D1))
    for k in (-2, 1, 3, 2048):
        with pytest.raises(DDQMCError) as e:
            g.set_graph_steps(k)
        assert e.value.code == -1
    g.set_graph_steps(10)
    g.set_graph_steps(0)
    for m in (-2, 2):
        with pytest.raises(DDQMCError) as e:
            g.set_heavy_fork(m)
        assert e.value.code == -1
    for q in (-1, 1025):
        with pytest.raises(DDQMCError) as e:
            g.set_tree_queue(q)
        assert e.value.code == -1
    for q in (-1, 3):
        with pytest.raises(DDQMCError) as e:
            g.set_loud_grid(q)
        assert e.value.code == -1
    g.set_loud_grid(2)
    g.set_loud_grid(1)
    g.set_tree_queue(1024)
    g.set_tree_queue(3)
    g.step(3)
    g.close()


def test_stage_times_sampled(dq):
    """Stage events on every k-th step: the step count and the stage layout
    (seal and histogram empty), and the same lists as without events."""
    from paper_1802_05931_amd import DDQMCError
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=20)
    a = dq.Solve(dq.make_params(**cfg))
    b = dq.Solve(dq.make_params(**cfg))
    with pytest.raises(DDQMCError) as e:
        b.set_profiling(-1)
    assert e.value.code == -1
    b.set_profiling(3)
    a.step(10)
    b.step(10)
    ms, n = b.stage_times()
    assert n == 4  # steps 0, 3, 6, 9 of the call
    assert ms["seal"] == 0.0 and ms["histogram"] == 0.0
    assert all(v >= 0.0 for v in ms.values()) and ms["loud"] > 0.0 and ms["merge"] > 0.0
    assert _same_list(a.walkers(), b.walkers())
    b.set_profiling(0)
    a.step(5)
    b.step(5)
    assert _same_list(a.walkers(), b.walkers())
    a.close()
    b.close()


def _churn_requests():
    rng = np.random.default_rng(7)
    lat = [(2, 2), (3, 3), (2, 6), (4, 4)]
    reqs = []
    for i in range(14):
        Lx, Ly = lat[i % 4]
        reqs.append(dict(params=dict(Lx=Lx, Ly=Ly, Jx=float(rng.uniform(0.6, 1.1)), Jy=1.0,
                                     Jz=float(rng.uniform(0.8, 1.2)),
                                     gamma=float(rng.uniform(1.2, 2.0)), dt=0.005, n_a=3,
                                     target_walkers=int(rng.integers(300, 3000)),
                                     initial_walkers=int(rng.integers(300, 3000)),
                                     shift_init=0.0, seed=11, solve_id=100 + i, n_equil=30),
                         steps=int(rng.integers(2, 9)) * 25))
    return reqs


@pytest.mark.parametrize("cap,gk,fork", [(0, 0, 0), (16, 0, 0), (16, 10, 0), (16, 10, 1)])
def test_pool_churn_equals_alone(dq, cap, gk, fork):
    """Continuous batching with churn: solves of four lattice shapes enter and
    leave a 5-slot pool between ticks (several admissions in one tick, slots
    reused, the buffers grown during entering steps when the capacity starts
    tiny; with gk > 0 the ticks run as k-step graphs, re-captured after each
    growth; with fork = 1 the large entries run on the second stream); each
    solve's list when it leaves equals the same solve run alone."""
    from paper_1802_05931_amd import DDQMCError
    reqs = _churn_requests()
    pool = dq.Pool(slots=5, max_sites=16, capacity_hint=cap)
    pool.set_heavy_fork(fork)
    if gk:
        pool.set_graph_steps(gk)
    queue = list(range(len(reqs)))
    active, done = {}, {}
    ticks = 0
    while queue or active:
        while queue:
            try:
                s = pool.admit(dq.make_params(**reqs[queue[0]]["params"]))
            except DDQMCError as e:
                assert e.code == -7
                break
            active[s] = queue.pop(0)
        pool.step(25)
        ticks += 1
        for s in list(active):
            i = active[s]
            st = pool.scalars(s)["step"]
            if st >= reqs[i]["steps"]:
                done[i] = (st, pool.walkers(s), pool.scalars(s))
                pool.retire(s)
                del active[s]
        assert ticks < 200
    pool.close()
    print(f"  churn: {len(done)} solves served in {ticks} ticks", flush=True)
    for i, (st, lst, sc) in done.items():
        g = dq.Solve(dq.make_params(**reqs[i]["params"]))
        g.step(st)
        assert _same_list(g.walkers(), lst), i
        assert g.scalars() == sc, i
        g.close()


def test_int32_overflow_reports_and_keeps_state(dq):
    from paper_1802_05931_amd import DDQMCError
    g = dq.Solve(dq.make_params(Lx=2, Ly=2, dt=0.5, shift_init=-3.0, target_walkers=2 ** 62,
                                initial_walkers=2 ** 31 - 10))
    before = g.walkers()
    with pytest.raises(DDQMCError) as e:
        g.step(5)
    assert e.value.code == -4
    after = g.walkers()
    assert g.scalars()["step"] == 0 and _same_list(before, after)
    g.close()


def test_invalid_parameters(dq):
    from paper_1802_05931_amd import DDQMCError
    for bad in [dict(Lx=1), dict(Lx=8, Ly=8), dict(dt=0.0), dict(gamma=-1.0), dict(n_a=-1),
                dict(initial_walkers=0), dict(initial_walkers=2 ** 31), dict(is_p=-1.0)]:
        with pytest.raises(DDQMCError) as e:
            dq.Solve(dq.make_params(**bad))
        assert e.value.code == -1


@pytest.mark.parametrize("extra", [dict(), dict(hx=0.1, hy=-0.05), dict(flags=2)],
                         ids=["plain", "field", "per_walker"])
def test_checkpoint_resume_bit_exact(dq, extra):
    """A handle restored from a checkpoint steps on exactly as the one it was
    taken from, for each sampler (the random streams are keyed on the
    configuration and the step, both in the checkpoint)."""
    cfg = dict(workloads.d2(0.6), target_walkers=5000, **extra)
    a = dq.Solve(dq.make_params(**cfg))
    a.step(300)
    blob = a.get_state()
    a.step(200)
    b = dq.Solve(dq.make_params(**cfg))
    b.set_state(blob)
    b.step(200)
    assert _same_list(a.walkers(), b.walkers())
    assert a.scalars() == b.scalars()


def test_full_size_4x4_window(dq, orc):
    """The 4x4 workload at full size: the GPU steps it until its list is steady
    (about 1.07e7 entries after some 14,500 steps, as the benchmark times it),
    at which size the list capacity is above 2^23 entries, so the large-entry
    kernel runs on the second stream beside the loud kernel, as in the timed
    steps; then two steps from that snapshot are checked against the oracle
    (DDQMC_D3_WINDOW steps, if set: 50 make the window that also times the
    oracle on this workload), and one more with merge tiles of 1024 positions
    (more than 8192 tiles: the merge offsets' coalesced round scan)."""
    cfg = dict(workloads.D3)
    g = dq.Solve(dq.make_params(**cfg))
    g.step(15000)
    keys, re, im = g.walkers()
    sc = g.scalars()
    _, cap = g.device_bytes()
    assert len(keys) > 10_000_000, len(keys)
    assert cap >= 1 << 23  # the fork's threshold (ddqmc_set_heavy_fork mode 0)
    counts = g.step_counts()[-1]
    assert counts[4] > 100 and counts[3] > 1_000_000  # heavy and loud entries at full size
    o = orc.Oracle(**cfg)
    o.set_list(keys, re, im)
    o.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
    print(f"  4x4 snapshot at step {sc['step']}: {len(keys)} entries", flush=True)
    del keys, re, im
    for i in range(int(os.environ.get("DDQMC_D3_WINDOW", "2"))):
        g.step(1)
        t0 = time.perf_counter()
        o.step(1)
        t_oracle = time.perf_counter() - t0
        assert _same_list(g.walkers(), o.get_list())
        assert g.scalars() == o.scalars()
        print(f"  4x4 window step {i + 1} bit-identical (oracle {t_oracle:.2f} s, "
              f"{o.size()} entries)", flush=True)
    g.set_tiles(8, 4)
    g.step(1)
    o.step(1)
    assert _same_list(g.walkers(), o.get_list())
    assert g.scalars() == o.scalars()
    assert sum(g.step_counts()[-1][:2]) > 8192 * 1024
    g.close()


def test_full_size_4x4_without_importance_sampling(dq, orc):
    """The 4x4 workload without importance sampling (p = 0) at full size: its
    steady list holds about 1.38e7 entries after some 8,500 steps (its two
    list buffers, 330 MB, no longer fit the 256 MB last-level cache) and a
    step emits about 1.9e6 records; two steps from that snapshot against the
    oracle."""
    cfg = dict(workloads.D3, is_p=0.0)
    g = dq.Solve(dq.make_params(**cfg))
    g.step(8500)
    keys, re, im = g.walkers()
    sc = g.scalars()
    assert len(keys) > 13_000_000, len(keys)
    assert g.step_counts()[-1][3] > 1_000_000  # loud entries at full size
    o = orc.Oracle(**cfg)
    o.set_list(keys, re, im)
    o.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
    print(f"  4x4 p = 0 snapshot at step {sc['step']}: {len(keys)} entries", flush=True)
    del keys, re, im
    for i in range(2):
        g.step(1)
        o.step(1)
        assert _same_list(g.walkers(), o.get_list())
        assert g.scalars() == o.scalars()
        print(f"  4x4 p = 0 window step {i + 1} bit-identical", flush=True)
    g.close()


def test_d1_full_run(dq, orc):
    """D1 (2x2) for all of its 10^4 steps, the series and accumulators included."""
    cfg = dict(workloads.D1)
    _compare_run(dq, orc, cfg, chunks=10, per=workloads.D1_STEPS // 10)


@pytest.mark.parametrize("jx", [0.6, 0.9, 1.1])
def test_d2_window_at_full_target(dq, orc, jx):
    """D2 (3x3) at its full target of 1e5 walkers, seed 0: the GPU runs 3000
    steps (past the growth phase), then the oracle follows a 1000-step window
    from that snapshot, compared every 250 steps."""
    cfg = dict(workloads.d2(jx))
    g = dq.Solve(dq.make_params(**cfg))
    g.step(3000)
    keys, re, im = g.walkers()
    sc = g.scalars()
    assert sc["mode"] == 1  # the shift varies: the target was reached
    o = orc.Oracle(**cfg)
    o.set_list(keys, re, im)
    o.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
    for c in range(4):
        g.step(250)
        o.step(250)
        assert _same_list(g.walkers(), o.get_list()), c
        assert g.scalars() == o.scalars()
        print(f"  3x3 Jx {jx}: step {o.scalars()['step']}, {len(o.get_list()[0])} entries ok",
              flush=True)
    g.close()


def test_d5_replicas_batch_equals_oracle(dq, orc):
    """Four of the 64 5x5 replicas of the batched workload (their own Jx,
    targets and solve ids), in one batch handle with 50-step graphs as the
    benchmark runs them, against the oracle run alone for each."""
    cfgs = workloads.d5_replicas()
    pick = [0, 21, 42, 63]
    b = dq.Batch([dq.make_params(**cfgs[i]) for i in pick])
    b.set_graph_steps(50)
    orcs = [orc.Oracle(**cfgs[i]) for i in pick]
    for c in range(3):
        b.step(100)
        for j, o in enumerate(orcs):
            o.step(100)
            assert _same_list(b.walkers(j), o.get_list()), (pick[j], c)
            assert b.scalars(j) == o.scalars(), pick[j]
        print(f"  5x5 replicas: {(c + 1) * 100} steps ok", flush=True)
    for j, o in enumerate(orcs):
        assert np.array_equal(b.series(j), o.series())
    b.close()


@pytest.mark.parametrize("sort_it,merge_it", [(4, 4), (4, 8), (8, 4), (16, 4), (16, 8)])
def test_tile_shapes_equal_the_oracle(dq, orc, sort_it, merge_it):
    """Every sort / merge tile shape the tuner may choose gives the oracle's lists
    (3x3 over several tiles; one step of a 5x5 list with 64-bit keys)."""
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=100)
    g = dq.Solve(dq.make_params(**cfg))
    g.set_tiles(sort_it, merge_it)
    assert g.tiles() == (sort_it, merge_it)
    o = orc.Oracle(**cfg)
    for _ in range(2):
        g.step(250)
        o.step(250)
        assert _same_list(g.walkers(), o.get_list())
        assert g.scalars() == o.scalars()
    assert np.array_equal(g.series(), o.series())
    g.close()
    keys, re, im = workloads.random_list(5, 5, 30000, 40, seed=31)
    c5 = dict(Lx=5, Ly=5, Jx=0.6, Jy=1.0, Jz=1.2, gamma=1.0, dt=0.01, n_a=3, is_p=0.5,
              target_walkers=2 ** 62, seed=78)
    g = dq.Solve(dq.make_params(**c5))
    g.set_tiles(sort_it, merge_it)
    o = orc.Oracle(**c5)
    g.set_walkers(keys, re, im)
    g.set_scalars(0.1, 1, 7, 10 ** 6)
    o.set_list(keys, re, im)
    o.set_scalars(0.1, 1, 7, 10 ** 6)
    g.step(1)
    o.step(1)
    assert _same_list(g.walkers(), o.get_list())
    g.close()


def test_tile_table_switches_shapes(dq, orc):
    """A tile table changes the shape as the list grows (between chunks of
    steps, with 10-step graphs re-captured for each shape): the oracle's lists."""
    cfg = dict(workloads.d2(0.6), target_walkers=20000, n_equil=60, capacity_hint=16)
    g = dq.Solve(dq.make_params(**cfg))
    g.set_graph_steps(10)
    g.set_tile_table([(0, 16, 4), (500, 4, 8), (3000, 8, 4)])
    o = orc.Oracle(**{k: v for k, v in cfg.items() if k != "capacity_hint"})
    seen = set()
    for _ in range(8):
        g.step(60)
        o.step(60)
        seen.add(g.tiles())
        assert _same_list(g.walkers(), o.get_list())
    assert len(seen) >= 2, seen
    assert g.scalars() == o.scalars()
    g.close()


@pytest.mark.parametrize("extra", [dict(), dict(hx=0.08, hy=-0.05), dict(flags=2)],
                         ids=["plain", "field", "per_walker"])
def test_32_sites(dq, orc, extra):
    """N = 32 (4x8): the configuration fills a 64-bit key and the slot field is
    empty (slot bits at position 64).  One step from a seeded random list at
    three counters, then a short run from the all-down state, each against the
    oracle bit for bit, for the plain, field and per-walker samplers."""
    keys, re, im = workloads.random_list(4, 8, 4000, 60, seed=32, even="hx" not in extra)
    cfg = dict(Lx=4, Ly=8, Jx=0.7, Jy=1.0, Jz=1.1, gamma=1.0, dt=0.01, n_a=3, is_p=0.5,
               target_walkers=2 ** 62, seed=78, **extra)
    g = dq.Solve(dq.make_params(**cfg))
    o = orc.Oracle(**cfg)
    for step in (0, 1, 12345):
        g.set_walkers(keys, re, im)
        g.set_scalars(0.1, 1, step, 10 ** 6)
        o.set_list(keys, re, im)
        o.set_scalars(0.1, 1, step, 10 ** 6)
        g.step(1)
        o.step(1)
        assert _same_list(g.walkers(), o.get_list()), step
        assert g.scalars() == o.scalars()
    g.close()
    run = dict(cfg, target_walkers=3000, initial_walkers=3000, shift_init=0.0, n_equil=20,
               dt=0.004)
    g = dq.Solve(dq.make_params(**run))
    o = orc.Oracle(**run)
    for _ in range(2):
        g.step(30)
        o.step(30)
        assert _same_list(g.walkers(), o.get_list())
        assert g.scalars() == o.scalars()
    assert np.array_equal(g.series(), o.series())
    g.close()
