"""The library's buffer-growth and workspace arithmetic, on the host (no GPU):
ddqmc_plan_growth (what a step that outgrew its buffers grows them to, when it
refuses) and ddqmc_workspace_query (the exact device bytes of a handle).

These pin the limits the kernels rely on: list and record capacities at most
0x7FF00000 entries each, so that list + records + a merge tile's rounding stay
below 2^32 and every 32-bit count, position and tile offset in the kernels is
exact; the record need of a failed step (fullest segment x 64 segments) taken
in 64 bits, so that a fill near 2^26 or above cannot wrap to a small need; and
growth refused, not attempted, when it would leave less than the memory
reserve free."""
import numpy as np
import pytest

MAX_CAP = 0x7FF00000
NSEG = 64
GiB = 1 << 30
OK, EINVAL, ENOMEM, ECAPACITY = 0, -1, -2, -3


@pytest.fixture(scope="module")
def dq():
    import os
    from paper_1802_05931_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    import paper_1802_05931_amd as m
    return m


def _plan(dq, cap_main, cap_sp, need_main, seg_need, ks=4, free=256 * GiB, total=288 * GiB,
          limit=0):
    return dq.plan_growth(cap_main, cap_sp, need_main, seg_need, ks, free, total, limit)


def test_no_need_keeps_the_capacities(dq):
    rc, nm, ns, b = _plan(dq, 1 << 20, 1 << 18, 0, 0)
    assert rc == OK and nm == 1 << 20 and ns == 1 << 18
    assert b >= 2 * nm * 12 + 2 * ns * 12


def test_short_capacities_grow_by_half_their_need(dq):
    rc, nm, ns, _ = _plan(dq, 1 << 20, 1 << 18, 3_000_000, 0)
    assert rc == OK and nm == 3_000_000 + 1_500_000 + 4096 and ns == 1 << 18
    rc, nm, ns, _ = _plan(dq, 1 << 20, 1 << 18, 0, 10_000)
    need = 10_000 * NSEG
    assert rc == OK and nm == 1 << 20
    assert ns >= need + need // 2 + 4096 and ns % NSEG == 0 and ns - (need + need // 2 + 4096) < NSEG


def test_the_largest_buffer_and_beyond(dq):
    rc, nm, ns, _ = _plan(dq, 1 << 30, 1 << 28, MAX_CAP, 0, ks=8, free=1 << 50, total=1 << 50)
    assert rc == OK and nm == MAX_CAP
    assert _plan(dq, 1 << 30, 1 << 28, MAX_CAP + 1, 0, free=1 << 50)[0] == ECAPACITY
    assert _plan(dq, 1 << 30, 1 << 28, 1 << 40, 0, free=1 << 50)[0] == ECAPACITY
    rc, nm, ns, _ = _plan(dq, 1 << 30, 1 << 28, 0, MAX_CAP // NSEG, free=1 << 50, total=1 << 50)
    assert rc == OK and ns == MAX_CAP


@pytest.mark.parametrize("seg_need", [1 << 26, (1 << 26) + 1, 1 << 27, (1 << 32) - 1, 1 << 40,
                                      (1 << 64) - 1])
def test_record_need_is_taken_in_64_bits(dq, seg_need):
    """seg_need x 64 wraps 32 bits from 2^26 on (2^26 x 64 = 2^32 would read as 0):
    every such need is above the largest buffer and must be refused."""
    assert _plan(dq, 1 << 20, 1 << 18, 0, seg_need, free=1 << 60, total=1 << 60)[0] == ECAPACITY


def test_capacity_ceiling(dq):
    rc, nm, _, _ = _plan(dq, 4096, 4096, 5000, 0, limit=20000)
    assert rc == OK and nm == 5000 + 2500 + 4096
    rc, nm, _, _ = _plan(dq, 4096, 4096, 19000, 0, limit=20000)
    assert rc == OK and nm == 20000
    assert _plan(dq, 4096, 4096, 20001, 0, limit=20000)[0] == ECAPACITY
    assert _plan(dq, 4096, 4096, 0, 20001 // NSEG + 1, limit=20000)[0] == ECAPACITY
    # a ceiling above the largest buffer is the largest buffer
    assert _plan(dq, 4096, 4096, MAX_CAP + 1, 0, limit=1 << 40, free=1 << 50)[0] == ECAPACITY


def test_memory_reserve(dq):
    """The new arena must leave max(4 GiB, total / 32) free."""
    rc, nm, ns, b = _plan(dq, 1 << 20, 1 << 18, 1 << 24, 0)
    assert rc == OK
    total = 288 * GiB
    reserve = max(4 * GiB, total // 32)
    assert _plan(dq, 1 << 20, 1 << 18, 1 << 24, 0, free=b + reserve, total=total)[0] == OK
    assert _plan(dq, 1 << 20, 1 << 18, 1 << 24, 0, free=b + reserve - 1,
                 total=total)[0] == ENOMEM
    small = 64 * GiB  # a reserve of 4 GiB on a small device
    assert _plan(dq, 1 << 20, 1 << 18, 1 << 24, 0, free=b + 4 * GiB, total=small)[0] == OK
    assert _plan(dq, 1 << 20, 1 << 18, 1 << 24, 0, free=b + 4 * GiB - 1,
                 total=small)[0] == ENOMEM


def test_growth_keeps_every_32_bit_position_exact(dq):
    """Over a sweep of needs up to the largest buffer: the grown capacities cover
    the need, stay at most MAX_CAP, and list + records + a merge tile's rounding
    (2047 positions) stays below 2^32."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        cm = int(rng.integers(4096, MAX_CAP))
        cs = int(rng.integers(4096, MAX_CAP)) // NSEG * NSEG
        nm_need = int(rng.integers(0, MAX_CAP + 1)) if rng.random() < 0.7 else 0
        sn = int(rng.integers(0, MAX_CAP // NSEG + 1)) if rng.random() < 0.7 else 0
        ks = 4 if rng.random() < 0.5 else 8
        rc, nm, ns, b = _plan(dq, cm, cs, nm_need, sn, ks=ks, free=1 << 50, total=1 << 50)
        assert rc == OK
        assert nm >= max(cm, nm_need) and nm <= MAX_CAP
        assert ns >= max(cs, sn * NSEG) and ns <= MAX_CAP and ns % NSEG == 0
        assert ns // NSEG >= sn
        assert nm + ns + 2047 < 1 << 32
        assert b >= 2 * nm * (ks + 8) + 2 * ns * (ks + 8) and b % 256 == 0


def test_invalid_key_size(dq):
    assert _plan(dq, 4096, 4096, 0, 0, ks=16)[0] == EINVAL


def test_workspace_query_is_the_layout(dq):
    p4 = dq.make_params(**dict(Lx=4, Ly=4))
    p5 = dq.make_params(**dict(Lx=5, Ly=5))
    prev = 0
    for cap in (4096, 10000, 1 << 20, 1 << 24):
        b4 = dq.workspace_query(p4, cap)
        b5 = dq.workspace_query(p5, cap)
        # lists (twice), records (twice, a quarter of the list), loud list and queues
        assert b4 >= 2 * cap * 12 + 2 * (cap // 4) * 12 + cap * (3 * 4 + 4 + 8)
        assert b5 >= 2 * cap * 16 + 2 * (cap // 4) * 16 + cap * (3 * 4 + 8 + 8)
        assert b5 > b4 > prev and b4 % 256 == 0
        prev = b4
    # below the smallest capacity the smallest is used
    assert dq.workspace_query(p4, 1) == dq.workspace_query(p4, 4096)
    with pytest.raises(dq.DDQMCError):
        dq.workspace_query(p4, -1)
