"""Pin of the oracle's annihilation (Sec. III.C, the third rule: walkers of
opposite sign on one configuration cancel) against a brute-force sum per
configuration in a Python dictionary.  Random lists and contributions over
small key spaces, so that keys repeat, totals cancel and list entries vanish;
keys with the top bit set (unsigned order); the empty cases; the int32 range
of the new values."""
import numpy as np
import pytest


def _brute(ck, cr, ci, keys, pr, pi):
    tot = {}
    for k, r, i in zip(keys.tolist(), pr.tolist(), pi.tolist()):
        tot[k] = [r, i]
    for k, r, i in zip(ck.tolist(), cr.tolist(), ci.tolist()):
        v = tot.setdefault(k, [0, 0])
        v[0] += r
        v[1] += i
    return sorted((k, r, i) for k, (r, i) in tot.items() if r != 0 or i != 0)


def _rows(out):
    return list(zip(*(a.tolist() for a in out)))


def _keys(rng, space, n):
    if space is None:  # the whole 64-bit range, top bit included
        return rng.integers(0, 2 ** 64 - 1, n, dtype=np.uint64, endpoint=True)
    return rng.integers(0, space, n).astype(np.uint64)


@pytest.mark.parametrize("seed", range(16))
def test_annihilation_equals_a_sum_per_configuration(orc, seed):
    rng = np.random.default_rng(seed)
    space = [8, 64, 1 << 40, None][seed % 4]
    keys = np.unique(_keys(rng, space, int(rng.integers(0, 60))))
    pr = rng.integers(-3, 4, len(keys))
    pi = rng.integers(-3, 4, len(keys))
    ncon = int(rng.integers(0, 200))
    ck = _keys(rng, space, ncon)
    if space is None and len(keys) and ncon:  # some contributions on list keys
        ck[: ncon // 2] = rng.choice(keys, ncon // 2)
    cr = rng.integers(-3, 4, ncon)
    ci = rng.integers(-3, 4, ncon)
    got = _rows(orc.annihilate(ck, cr, ci, keys, pr, pi))
    assert got == _brute(ck, cr, ci, keys, pr, pi)
    assert all(r != 0 or i != 0 for _, r, i in got)


def test_annihilation_empty_cases(orc):
    e = np.zeros(0, np.uint64)
    z = np.zeros(0, np.int64)
    assert _rows(orc.annihilate(e, z, z, e, z, z)) == []
    keys = np.array([1, 5, 9], np.uint64)
    assert _rows(orc.annihilate(e, z, z, keys, np.array([2, 0, -1]), np.array([0, 0, 3]))) == \
        [(1, 2, 0), (9, -1, 3)]  # an entry moved to zero by its own death is gone
    ck = np.array([7, 3, 7, 3], np.uint64)
    assert _rows(orc.annihilate(ck, np.array([1, 2, -1, 0]), np.array([0, 1, 0, 0]), e, z, z)) == \
        [(3, 2, 1)]


def test_annihilation_int32_range(orc):
    keys = np.array([4], np.uint64)
    top = 2 ** 31 - 1
    zero = np.array([0], np.int64)
    assert _rows(orc.annihilate(keys, zero, zero, keys, np.array([top]), np.array([-top]))) == \
        [(4, top, -top)]
    for pr, pi, cr, ci in [(top, 0, 1, 0), (0, -top, 0, -1), (-top, 0, -1, 0)]:
        with pytest.raises(orc.OracleError) as e:
            orc.annihilate(keys, np.array([cr]), np.array([ci]), keys, np.array([pr]),
                           np.array([pi]))
        assert e.value.code == orc.EOVERFLOW
    # a total back inside the range is kept
    assert _rows(orc.annihilate(np.array([4, 4], np.uint64), np.array([1, -1]), zero.repeat(2),
                                keys, np.array([top]), zero)) == [(4, top, 0)]
