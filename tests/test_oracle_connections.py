"""The oracle's Liouvillian elements seen from a parent configuration, pinned to
the Kronecker-form Liouvillian of Sec. III.C with the importance-sampling
weights of Sec. IV.B.

For every configuration of 2x2 and 2x3 the oracle's enumerated children with
their element values, and its diagonal element (d_re, d_im), must equal the
corresponding column of the sparse Kronecker matrix.  For 3x3 and 4x4 random
columns are compared with a per-column build from the sparse H.
"""
import numpy as np
import pytest

from oracle import exact

PARAMS = dict(Jx=0.9, Jy=1.0, Jz=1.3, gamma=0.8)


def _oracle_column(orc, Lx, Ly, l, m, S, is_p, hx=0.0, hy=0.0):
    p = orc.make_params(Lx=Lx, Ly=Ly, is_p=is_p, hx=hx, hy=hy, **PARAMS)
    ck, cb, re, im, dr, di = orc.connections(p, l, m, S)
    out = {}
    for a, b, x, y in zip(ck.tolist(), cb.tolist(), re.tolist(), im.tolist()):
        assert (a, b) not in out, "child listed twice"
        out[(a, b)] = complex(x, y)
    return out, complex(dr, di)


def _compare(ora, diag, col, l, m):
    exp = {k: v for k, v in col.items() if abs(v) > 0}
    d_exp = exp.pop((l, m), 0)
    assert set(k for k, v in ora.items() if v != 0) == set(exp), (l, m)
    for k, v in exp.items():
        assert abs(ora[k] - v) <= 1e-15 * max(1.0, abs(v)), (l, m, k, ora[k], v)
    assert abs(diag - d_exp) <= 1e-14 * max(1.0, abs(d_exp)), (l, m, diag, d_exp)


@pytest.mark.parametrize("Lx,Ly,is_p,S", [(2, 2, 0.0, 0.0), (2, 2, 1.5, 0.37), (2, 3, 1.5, -0.2)])
def test_every_column_small_lattices(orc, Lx, Ly, is_p, S):
    N = Lx * Ly
    D = 2 ** N
    L = exact.liouvillian(Lx, Ly, PARAMS["Jx"], PARAMS["Jy"], PARAMS["Jz"], PARAMS["gamma"],
                          S=S, is_p=is_p).tocsc()
    for m in range(D):
        for l in range(D):
            c = L[:, m * D + l]
            col = {(int(i) % D, int(i) // D): v for i, v in zip(c.indices, c.data)}
            ora, diag = _oracle_column(orc, Lx, Ly, l, m, S, is_p)
            _compare(ora, diag, col, l, m)


@pytest.mark.parametrize("Lx,Ly,ncols", [(3, 3, 60), (4, 4, 25), (2, 6, 40)])
def test_random_columns_larger_lattices(orc, Lx, Ly, ncols):
    N = Lx * Ly
    rng = np.random.default_rng(Lx * 10 + Ly)
    for _ in range(ncols):
        l = int(rng.integers(0, 2 ** N))
        m = int(rng.integers(0, 2 ** N))
        if rng.random() < 0.3:
            m = l
        if rng.random() < 0.3:  # one bond away: exercises the to-diagonal class
            bl = exact.bonds(Lx, Ly)
            a, b = bl[int(rng.integers(0, len(bl)))]
            m = l ^ (1 << a) ^ (1 << b)
        col = exact.column(Lx, Ly, PARAMS["Jx"], PARAMS["Jy"], PARAMS["Jz"], PARAMS["gamma"],
                           l, m, S=0.11, is_p=1.5)
        ora, diag = _oracle_column(orc, Lx, Ly, l, m, 0.11, 1.5)
        _compare(ora, diag, col, l, m)


def test_oracle_bond_order_matches_exact(orc):
    for Lx, Ly in [(2, 2), (3, 3), (4, 4), (2, 6), (5, 5), (4, 8)]:
        assert orc.bonds(Lx, Ly) == exact.bonds(Lx, Ly)


@pytest.mark.parametrize("Lx,Ly,is_p,S,hx,hy", [(2, 2, 0.0, 0.0, 0.3, 0.0),
                                               (2, 2, 1.5, 0.37, 0.0, -0.2),
                                               (2, 3, 0.8, -0.2, 0.15, 0.25)])
def test_every_column_with_field(orc, Lx, Ly, is_p, S, hx, hy):
    """With the in-plane field (Sec. V.B): the single-flip children carry both a
    real and an imaginary element part, each configuration of either parity."""
    N = Lx * Ly
    D = 2 ** N
    L = exact.liouvillian(Lx, Ly, PARAMS["Jx"], PARAMS["Jy"], PARAMS["Jz"], PARAMS["gamma"],
                          S=S, is_p=is_p, hx=hx, hy=hy).tocsc()
    for m in range(D):
        for l in range(D):
            c = L[:, m * D + l]
            col = {(int(i) % D, int(i) // D): v for i, v in zip(c.indices, c.data)}
            ora, diag = _oracle_column(orc, Lx, Ly, l, m, S, is_p, hx, hy)
            _compare(ora, diag, col, l, m)


def test_random_columns_with_field_4x4(orc):
    rng = np.random.default_rng(44)
    for _ in range(25):
        l = int(rng.integers(0, 2 ** 16))
        m = int(rng.integers(0, 2 ** 16))
        r = rng.random()
        if r < 0.3:
            m = l
        elif r < 0.6:  # one flip away: the field's to-diagonal class
            m = l ^ (1 << int(rng.integers(0, 16)))
        col = exact.column(4, 4, PARAMS["Jx"], PARAMS["Jy"], PARAMS["Jz"], PARAMS["gamma"],
                           l, m, S=0.11, is_p=1.5, hx=0.12, hy=-0.07)
        ora, diag = _oracle_column(orc, 4, 4, l, m, 0.11, 1.5, 0.12, -0.07)
        _compare(ora, diag, col, l, m)
