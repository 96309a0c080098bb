"""Pins of the exact Liouvillian / steady-state solver (the reference the DDQMC
estimators are checked against, Sec. V "solving the linear system").

* The Kronecker form of Sec. III.C equals the master equation of Sec. III.A applied
  directly to every basis operator |l><m| (dense matrix products).
* The steady state has zero residual, unit trace, is Hermitian and positive.
* Closed forms: Jx = Jy makes |dn..dn> an eigenstate of H with no up spin, so the
  steady state is |dn..dn><dn..dn| (M_z = -1); J = 0 likewise.
* At zero field the parity selection rule forces <sigma^x> = <sigma^y> = 0; with
  the in-plane field of Sec. V.B they respond linearly at small field, along
  and (through the anisotropy) across the field.
* Trace preservation: the diagonal rows of L sum to zero.
"""
import numpy as np
import pytest

from oracle import exact


@pytest.mark.parametrize("Lx,Ly", [(2, 2)])
def test_kronecker_equals_master_equation(Lx, Ly):
    Ld = exact.liouvillian_direct(Lx, Ly, 0.9, 1.0, 1.3, 0.7)
    Lk = exact.liouvillian(Lx, Ly, 0.9, 1.0, 1.3, 0.7).toarray()
    assert np.abs(Ld - Lk).max() < 1e-14


def test_kronecker_action_on_random_rho_2x3():
    Lx, Ly = 2, 3
    D = 2 ** (Lx * Ly)
    rng = np.random.default_rng(3)
    rho = rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D))
    H = exact.hamiltonian(Lx, Ly, 0.7, 1.0, 1.1).toarray()
    gamma = 0.8
    direct = -1j * (H @ rho - rho @ H)
    for F in exact.jump_ops(Lx, Ly):
        F = F.toarray()
        FdF = F.conj().T @ F
        direct += gamma * (F @ rho @ F.conj().T - 0.5 * (FdF @ rho + rho @ FdF))
    L = exact.liouvillian(Lx, Ly, 0.7, 1.0, 1.1, gamma)
    kron = (L @ rho.reshape(-1, order="F")).reshape((D, D), order="F")
    assert np.abs(kron - direct).max() < 1e-12


def test_trace_preservation_rows():
    L = exact.liouvillian(2, 2, 0.9, 1.0, 1.0, 1.0).toarray()
    D = 16
    diag_rows = [l * D + l for l in range(D)]
    assert np.abs(L[diag_rows].sum(axis=0)).max() < 1e-14


def test_bond_counts():
    assert len(exact.bonds(2, 2)) == 4
    assert len(exact.bonds(3, 3)) == 18
    assert len(exact.bonds(4, 4)) == 32
    assert len(exact.bonds(2, 6)) == 18
    assert len(exact.bonds(5, 5)) == 50


@pytest.mark.parametrize("Lx,Ly,Jx", [(2, 2, 0.9), (2, 3, 0.6)])
def test_ness_properties(Lx, Ly, Jx):
    rho = exact.ness(Lx, Ly, Jx, 1.0, 1.0, 1.0)
    D = rho.shape[0]
    L = exact.liouvillian(Lx, Ly, Jx, 1.0, 1.0, 1.0)
    res = L @ rho.reshape(-1, order="F")
    assert np.abs(res).max() < 1e-11
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-11
    ev = np.linalg.eigvalsh(0.5 * (rho + rho.conj().T))
    assert ev.min() > -1e-11
    obs = exact.observables(rho, Lx, Ly)
    assert abs(obs["mx"]) < 1e-13 and abs(obs["my"]) < 1e-13
    assert -1.0 < obs["mz"] < 0.0
    assert D == 2 ** (Lx * Ly)


@pytest.mark.parametrize("Jx,Jy", [(0.8, 0.8), (0.0, 0.0)])
def test_ness_closed_form_all_down(Jx, Jy):
    rho = exact.ness(2, 2, Jx, Jy, 1.0, 1.0)
    expected = np.zeros_like(rho)
    expected[0, 0] = 1.0
    assert np.abs(rho - expected).max() < 1e-12
    assert exact.observables(rho, 2, 2)["mz"] == pytest.approx(-1.0, abs=1e-14)


def test_single_spin_relaxation_closed_form():
    """A lone decaying spin (no bonds contribute when J = 0): the coherence
    |up><dn| decays at gamma/2 and the up population at gamma."""
    gamma = 1.7
    L = exact.liouvillian(2, 2, 0.0, 0.0, 0.0, gamma).toarray()
    D = 16
    up0 = 1  # site 0 up, others down
    col = L[:, up0 * D + up0]
    assert col[up0 * D + up0] == pytest.approx(-gamma)
    assert col[0] == pytest.approx(gamma)
    coh = L[:, 0 * D + up0]   # rho_{up0, 0}
    assert coh[0 * D + up0] == pytest.approx(-gamma / 2)


def test_pauli_y_convention():
    """sigma^y in the (down, up) basis of the bit: sigma^y |up> = i |down> and
    sigma^y |down> = -i |up>, so <down|sigma^y|up> = i; and it squares to 1 and
    anticommutes with sigma^x, with sigma^x sigma^y = i sigma^z."""
    assert exact.SY[0, 1] == 1j and exact.SY[1, 0] == -1j
    assert np.allclose(exact.SY @ exact.SY, np.eye(2))
    assert np.allclose(exact.SX @ exact.SY, 1j * exact.SZ)


@pytest.mark.parametrize("hx,hy", [(0.3, 0.0), (0.0, -0.2), (0.15, 0.25)])
def test_kronecker_with_field_equals_master_equation(hx, hy):
    """With the in-plane field of Sec. V.B in H (hx sigma^x + hy sigma^y per site)."""
    Ld = exact.liouvillian_direct(2, 2, 0.9, 1.0, 1.3, 0.7, hx=hx, hy=hy)
    Lk = exact.liouvillian(2, 2, 0.9, 1.0, 1.3, 0.7, hx=hx, hy=hy).toarray()
    assert np.abs(Ld - Lk).max() < 1e-14
    # the field term is H's only part between configurations one flip apart:
    # <up|hx sigma^x + hy sigma^y|dn> = hx - i hy = h e^{-i theta}
    H = exact.hamiltonian(2, 2, 0.9, 1.0, 1.3, hx, hy).toarray()
    assert H[0b0001, 0b0000] == hx - 1j * hy and H[0b0000, 0b0001] == hx + 1j * hy


def test_field_breaks_parity_and_gives_linear_response():
    """The field makes the transverse magnetisation nonzero.  As for one driven
    spin decaying to |dn> (the field resonant, no detuning), a field along x
    gives <sigma^y> and no <sigma^x>: the response tensor is off-diagonal, and
    a field along y gives mostly <sigma^x>, of opposite sign.  At small h the
    response is linear (M(2h) = 2 M(h) up to 0.5% at h = 0.01)."""
    Lx, Ly = 2, 2
    r1 = exact.observables(exact.ness(Lx, Ly, 0.9, 1.0, 1.0, 1.0, hx=0.01), Lx, Ly)
    r2 = exact.observables(exact.ness(Lx, Ly, 0.9, 1.0, 1.0, 1.0, hx=0.02), Lx, Ly)
    assert abs(r1["mx"]) < 1e-14 and r1["my"] > 1e-2
    assert abs(r2["my"] / r1["my"] - 2.0) < 1e-2
    ry = exact.observables(exact.ness(Lx, Ly, 0.9, 1.0, 1.0, 1.0, hy=0.01), Lx, Ly)
    assert ry["mx"] < -1e-2 and abs(ry["my"]) > 1e-3
    rho = exact.ness(Lx, Ly, 0.9, 1.0, 1.0, 1.0, hx=0.2, hy=0.1)
    L = exact.liouvillian(Lx, Ly, 0.9, 1.0, 1.0, 1.0, hx=0.2, hy=0.1)
    assert np.abs(L @ rho.reshape(-1, order="F")).max() < 1e-12
    assert abs(np.trace(rho) - 1) < 1e-12 and np.abs(rho - rho.conj().T).max() < 1e-12
    assert np.linalg.eigvalsh(rho).min() > -1e-12


def test_long_time_limit_equals_the_direct_solve():
    """The steady state by integrating the master equation to its long-time
    limit (the route used for 3x3, where the direct sparse solve fills in too
    much) equals the direct solve of L rho = 0, Tr rho = 1 on 2x3."""
    rho_d = exact.ness(2, 3, 0.6, 1.0, 1.0, 1.0)
    rho_e, res = exact.ness_evolve(2, 3, 0.6, 1.0, 1.0, 1.0)
    assert res < 1e-12
    assert np.abs(rho_e - rho_d).max() < 1e-9
    od, oe = exact.observables(rho_d, 2, 3), exact.observables(rho_e, 2, 3)
    assert all(abs(od[k] - oe[k]) < 1e-9 for k in od)


def test_golden_3x3_steady_states():
    """tests/golden/ness_3x3.json (written by make_ness_3x3.py from the same
    integration) holds converged 3x3 steady states: residual below 1e-12, and
    the physics the 2x3 lattice shows too (M_z in (-1, 0), and closer to -1
    the nearer Jx is to Jy, where the all-down state is exact)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ness_3x3.json")))
    by = {s["Jx"]: s for s in g["states"]}
    assert set(by) == {0.6, 0.9, 1.1}
    for s in by.values():
        assert s["residual"] < 1e-12 and -1.0 < s["mz"] < 0.0
        assert s["mx"] == 0.0 and s["my"] == 0.0
    assert by[0.6]["mz"] > by[0.9]["mz"]
