"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no part of the method's arithmetic: it only states the
workload parameters (lattice, couplings, walker counts, step counts) and draws
seeded random walker lists and serving/batch parameter sets.  Both the CPU
oracle and the GPU library are driven from here.

Workload shapes follow the paper's runs: 2x2, 3x3 and 4x4 periodic dissipative
XYZ lattices (Sec. V), 10^6-10^8 walkers (captions of the initiator and
occupied-element figures), importance-sampling p = 1.5 (occupied-element figure).
No dataset is involved; the physics run is the workload.
"""
import numpy as np

# parameter dictionaries use the field names of the C parameter structs
D1 = dict(Lx=2, Ly=2, Jx=0.9, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.01, n_a=3,
          target_walkers=1000, initial_walkers=100, is_p=0.0, shift_damping=0.05,
          shift_init=-0.5, seed=0, solve_id=0, n_equil=1000)
D1_STEPS = 10000


def d2(Jx=0.9, seed=0):
    return dict(Lx=3, Ly=3, Jx=Jx, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.005, n_a=3,
                target_walkers=100000, initial_walkers=100, is_p=0.0, shift_damping=0.05,
                shift_init=-0.5, seed=seed, solve_id=0, n_equil=4000)


D2_STEPS = 20000

# 4x4, importance sampling p = 1.5, started at the target on |dn..dn><dn..dn|
D3 = dict(Lx=4, Ly=4, Jx=0.9, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.002, n_a=3,
          target_walkers=10_000_000, initial_walkers=10_000_000, is_p=1.5,
          shift_damping=0.05, shift_init=0.0, seed=0, solve_id=0, n_equil=1000)
D3_STEPS = 5000


def d5_replicas(count=64, t_lo=1e3, t_hi=2e4):
    """64 independent 5x5 replicas, Jx spread evenly over [0.5, 1.2], targets
    log-uniform in [t_lo, t_hi] from default_rng(5).  Under population control
    of the diagonal weight alone, the off-diagonal population of a 5x5 replica
    keeps growing (the oracle: about x1.6 per 100 steps at target 2e3, x2.4 at
    target 2e4, p = 0, Jx = 0.5), so targets of 1e5-2e6 would outgrow the device
    within a few hundred steps; the default range is that one divided by 100."""
    rng = np.random.default_rng(5)
    targets = np.exp(rng.uniform(np.log(t_lo), np.log(t_hi), count)).astype(np.int64)
    out = []
    for r in range(count):
        out.append(dict(Lx=5, Ly=5, Jx=0.5 + 0.7 * r / max(count - 1, 1), Jy=1.0, Jz=1.0,
                        gamma=1.0, dt=0.002, n_a=3, target_walkers=int(targets[r]),
                        initial_walkers=int(targets[r]), is_p=0.0, shift_damping=0.05,
                        shift_init=0.0, seed=0, solve_id=r, n_equil=100))
    return out


D4_LATTICES = ((2, 2), (3, 3), (4, 4), (2, 6))


def d4_requests(count=512, rate=20.0, seed=20181802, t_lo=1e3, t_hi=1e5):
    """Serving stream: Poisson arrivals at ``rate`` per second, lattices uniform over
    2x2/3x3/4x4/2x6, Jx ~ U[0.5,1.2], Jz ~ U[0.8,1.2], gamma ~ U[0.5,2], dt 0.005,
    target walkers log-uniform in [t_lo, t_hi].  At small gamma a 4x4 or 2x6 list
    holds far more entries than its diagonal target (the oracle: 1.2e7 entries
    after 250 steps for target 1e5 at gamma 0.5), so the default upper target is
    1e5 rather than 1e6."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        Lx, Ly = D4_LATTICES[rng.integers(0, len(D4_LATTICES))]
        target = int(np.exp(rng.uniform(np.log(t_lo), np.log(t_hi))))
        out.append(dict(arrival=float(t[i]),
                        params=dict(Lx=int(Lx), Ly=int(Ly), Jx=float(rng.uniform(0.5, 1.2)),
                                    Jy=1.0, Jz=float(rng.uniform(0.8, 1.2)),
                                    gamma=float(rng.uniform(0.5, 2.0)), dt=0.005, n_a=3,
                                    target_walkers=target, initial_walkers=target, is_p=0.0,
                                    shift_damping=0.05, shift_init=0.0, seed=20181802,
                                    solve_id=i, n_equil=400)))
    return out


def random_list(Lx, Ly, n_entries, max_pop, seed, even=True, hermitian=False,
                include_diag0=True):
    """Sorted unique configuration keys (ket << N | bra) with nonzero random integer
    (re, im) populations in [-max_pop, max_pop].  ``even`` keeps
    popcount(ket)+popcount(bra) even.  ``hermitian`` makes the list closed under
    (ket, bra) -> (bra, ket) with conjugate populations and real diagonals."""
    N = Lx * Ly
    rng = np.random.default_rng(seed)
    D = 1 << N
    keys = set()
    if include_diag0:
        keys.add(0)
    while len(keys) < n_entries:
        l = int(rng.integers(0, D))
        m = int(rng.integers(0, D))
        if even and (bin(l).count("1") + bin(m).count("1")) % 2:
            continue
        keys.add((l << N) | m)
        if hermitian:
            keys.add((m << N) | l)
    keys = np.array(sorted(keys), dtype=np.uint64)
    n = len(keys)
    re = rng.integers(-max_pop, max_pop + 1, n).astype(np.int32)
    im = rng.integers(-max_pop, max_pop + 1, n).astype(np.int32)
    if hermitian:
        pos = {int(k): i for i, k in enumerate(keys)}
        for i, k in enumerate(keys):
            k = int(k)
            l, m = k >> N, k & (D - 1)
            j = pos[(m << N) | l]
            if l == m:
                im[i] = 0
            elif i < j:
                re[j] = re[i]
                im[j] = -im[i]
    zero = (re == 0) & (im == 0)
    re[zero] = 1
    return keys, re, im
