"""Exact Liouvillian and steady state of the dissipative XYZ lattice.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is built from 2x2 spin matrices with Kronecker products, with no
bit tricks, so that it is an independent check of the walker step:

* the model of Sec. V: H = sum over nearest-neighbour bonds of
  Jx Sx Sx + Jy Sy Sy + Jz Sz Sz with S = sigma/2, plus the in-plane field of
  Sec. V.B, sum over sites of h (cos theta sigma^x + sin theta sigma^y) =
  hx sigma^x + hy sigma^y, jump operator S^- per site at rate gamma, on a
  periodic Lx x Ly lattice;
* the vectorised shifted Liouvillian of Sec. III.C (column stacking):
  L = -i(1 (x) H - H^T (x) 1) - S 1 (x) 1
      + sum_k gamma/2 (2 F_k^* (x) F_k - 1 (x) F_k^dag F_k - F_k^T F_k^* (x) 1);
* the importance-sampled element form of Sec. IV.B: each off-diagonal element
  from parent (l,m) to child (i,j) is multiplied by w_ij / w_lm with
  w = e^{-p} off the diagonal and 1 on it;
* the steady state as the null vector of L with unit trace ("solving the linear
  system", Sec. V), and observables Tr(rho O) (Sec. III.A, Sec. V.A); for
  lattices where the direct sparse solve fills in too much (3x3), the
  steady state as the long-time limit of the master equation, integrated
  with the classical fourth-order Runge-Kutta rule.

Basis: state index = bitstring, bit s = 1 <=> spin up at site s = x + Lx*y.
The element rho_{lm} sits at vec index m*D + l (D = 2^N).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# single-site matrices in the basis (index 0 = down, index 1 = up)
SZ = np.array([[-1.0, 0.0], [0.0, 1.0]], dtype=complex)
SX = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=complex)
SY = np.array([[0.0, 1j], [-1j, 0.0]], dtype=complex)   # sigma_y|up> = i|down>
SM = np.array([[0.0, 1.0], [0.0, 0.0]], dtype=complex)   # sigma^- = |down><up|


def bonds(Lx, Ly):
    """Unique unordered nearest-neighbour pairs of the periodic lattice, listed
    as right bonds by origin site, then up bonds by origin site."""
    seen = set()
    right, up = [], []
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            r = (x + 1) % Lx + Lx * y
            if frozenset((s, r)) not in seen and r != s:
                seen.add(frozenset((s, r)))
                right.append((s, r))
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            u = x + Lx * ((y + 1) % Ly)
            if frozenset((s, u)) not in seen and u != s:
                seen.add(frozenset((s, u)))
                up.append((s, u))
    return right + up


def site_op(op, s, N):
    """op acting on site s of N sites; site s is bit s of the index, so it is the
    (N-1-s)-th factor of the Kronecker product."""
    left = sp.identity(2 ** (N - 1 - s), dtype=complex, format="csr")
    right = sp.identity(2 ** s, dtype=complex, format="csr")
    return sp.kron(sp.kron(left, sp.csr_matrix(op)), right, format="csr")


def hamiltonian(Lx, Ly, Jx, Jy, Jz, hx=0.0, hy=0.0):
    N = Lx * Ly
    D = 2 ** N
    H = sp.csr_matrix((D, D), dtype=complex)
    ops = {s: (site_op(SX, s, N), site_op(SY, s, N), site_op(SZ, s, N)) for s in range(N)}
    for a, b in bonds(Lx, Ly):
        xa, ya, za = ops[a]
        xb, yb, zb = ops[b]
        H = H + 0.25 * (Jx * (xa @ xb) + Jy * (ya @ yb) + Jz * (za @ zb))
    for s in range(N):
        H = H + hx * ops[s][0] + hy * ops[s][1]
    return H.tocsr()


def jump_ops(Lx, Ly):
    N = Lx * Ly
    return [site_op(SM, s, N) for s in range(N)]


def liouvillian(Lx, Ly, Jx, Jy, Jz, gamma, S=0.0, is_p=0.0, hx=0.0, hy=0.0):
    """Sparse shifted Liouvillian in the Kronecker form, with importance-sampling
    factors applied to the off-diagonal elements."""
    N = Lx * Ly
    D = 2 ** N
    H = hamiltonian(Lx, Ly, Jx, Jy, Jz, hx, hy)
    I = sp.identity(D, dtype=complex, format="csr")
    L = -1j * (sp.kron(I, H) - sp.kron(H.T, I))
    for F in jump_ops(Lx, Ly):
        FdF = (F.conj().T @ F).tocsr()
        L = L + 0.5 * gamma * (2.0 * sp.kron(F.conj(), F) - sp.kron(I, FdF)
                               - sp.kron(F.T @ F.conj(), I))
    L = (L - S * sp.identity(D * D, dtype=complex)).tocoo()
    if is_p != 0.0:
        w = weights(N, is_p)
        data = L.data * np.where(L.row != L.col, w[L.row] / w[L.col], 1.0)
        L = sp.coo_matrix((data, (L.row, L.col)), shape=L.shape)
    return L.tocsc()


def weights(N, is_p):
    """w_lm = e^{-p} off the diagonal, 1 on it, at vec index m*D + l."""
    D = 2 ** N
    idx = np.arange(D * D)
    l = idx % D
    m = idx // D
    return np.where(l == m, 1.0, np.exp(-is_p))


def liouvillian_direct(Lx, Ly, Jx, Jy, Jz, gamma, hx=0.0, hy=0.0):
    """Dense Liouvillian built column by column from the master equation itself,
    L(|l><m|) = -i[H, |l><m|] + sum_k gamma (F |l><m| F^dag - {F^dag F, |l><m|}/2),
    with dense matrix products.  Small lattices only; used to pin the Kronecker
    form."""
    N = Lx * Ly
    D = 2 ** N
    H = hamiltonian(Lx, Ly, Jx, Jy, Jz, hx, hy).toarray()
    Fs = [F.toarray() for F in jump_ops(Lx, Ly)]
    L = np.zeros((D * D, D * D), dtype=complex)
    for m in range(D):
        for l in range(D):
            E = np.zeros((D, D), dtype=complex)
            E[l, m] = 1.0
            out = -1j * (H @ E - E @ H)
            for F in Fs:
                FdF = F.conj().T @ F
                out += gamma * (F @ E @ F.conj().T - 0.5 * (FdF @ E + E @ FdF))
            L[:, m * D + l] = out.reshape(-1, order="F")
    return L


def ness(Lx, Ly, Jx, Jy, Jz, gamma, hx=0.0, hy=0.0):
    """Steady state: L rho = 0 with Tr rho = 1.  One diagonal equation is replaced
    by the trace condition (the diagonal rows of L sum to zero because the
    evolution preserves the trace).  Without the field, restricted to the even
    sector popcount(l) + popcount(m) even, which the evolution from
    |dn..dn><dn..dn| never leaves; the field breaks that parity, and then the
    whole space is used."""
    N = Lx * Ly
    D = 2 ** N
    L = liouvillian(Lx, Ly, Jx, Jy, Jz, gamma, hx=hx, hy=hy)
    idx = np.arange(D * D)
    l = idx % D
    m = idx // D
    pc = np.array([bin(i).count("1") for i in range(D)])
    if hx == 0.0 and hy == 0.0:
        even = np.nonzero((pc[l] + pc[m]) % 2 == 0)[0]
    else:
        even = idx
    Le = L[even][:, even].tolil()
    diag_pos = np.nonzero(l[even] == m[even])[0]
    r = diag_pos[0]
    Le[r, :] = 0.0
    for j in diag_pos:
        Le[r, j] = 1.0
    b = np.zeros(len(even), dtype=complex)
    b[r] = 1.0
    x = spla.spsolve(Le.tocsc(), b)
    vec = np.zeros(D * D, dtype=complex)
    vec[even] = x
    return vec.reshape((D, D), order="F")


def ness_evolve(Lx, Ly, Jx, Jy, Jz, gamma, tau=0.05, tol=1e-12, t_max=200.0):
    """Steady state as the limit t -> infinity of d rho / dt = L rho, from the
    all-down state, in the even sector popcount(l) + popcount(m) even (the
    evolution never leaves it without a field): classical fourth-order
    Runge-Kutta steps of length tau until max |L rho| / max |rho| < tol.
    The trace is conserved by L; rho is returned with unit trace, and the
    relative residual reached."""
    N = Lx * Ly
    D = 2 ** N
    L = liouvillian(Lx, Ly, Jx, Jy, Jz, gamma)
    idx = np.arange(D * D)
    l = idx % D
    m = idx // D
    pc = np.array([bin(i).count("1") for i in range(D)])
    even = np.nonzero((pc[l] + pc[m]) % 2 == 0)[0]
    Le = L[even][:, even].tocsr()
    x = np.zeros(len(even), dtype=complex)
    x[np.nonzero(even == 0)[0][0]] = 1.0
    t = 0.0
    res = np.inf
    while t < t_max:
        for _ in range(100):
            k1 = Le @ x
            k2 = Le @ (x + 0.5 * tau * k1)
            k3 = Le @ (x + 0.5 * tau * k2)
            k4 = Le @ (x + tau * k3)
            x = x + (tau / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            t += tau
        res = np.abs(Le @ x).max() / np.abs(x).max()
        if res < tol:
            break
    vec = np.zeros(D * D, dtype=complex)
    vec[even] = x
    rho = vec.reshape((D, D), order="F")
    return rho / np.trace(rho), res


def observables(rho, Lx, Ly):
    """Per-site magnetisations and bond-averaged correlators, Tr(rho O)."""
    N = Lx * Ly
    tr = np.trace(rho).real
    out = {}
    for name, op in (("mx", SX), ("my", SY), ("mz", SZ)):
        tot = 0.0
        for s in range(N):
            O = site_op(op, s, N)
            tot += (O.multiply(rho.T)).sum().real   # Tr(rho O) = sum_ij rho_ij O_ji
        out[name] = tot / (N * tr)
    bl = bonds(Lx, Ly)
    for name, op in (("cxx", SX), ("cyy", SY), ("czz", SZ)):
        tot = 0.0
        for a, b in bl:
            O = site_op(op, a, N) @ site_op(op, b, N)
            tot += (O.multiply(rho.T)).sum().real
        out[name] = tot / (len(bl) * tr)
    return out


def vec_index(key, N):
    """Configuration key (ket << N) | bra  ->  vec index bra*D + ket."""
    D = 2 ** N
    key = np.asarray(key, dtype=np.uint64)
    l = (key >> np.uint64(N)).astype(np.int64)
    m = (key & np.uint64(D - 1)).astype(np.int64)
    return m * D + l


def one_step_expectation(keys, re, im, Lx, Ly, Jx, Jy, Jz, gamma, dt, S, is_p=0.0,
                         non_initiator=None, hx=0.0, hy=0.0):
    """Exact E[rho_{n+1} | rho_n] = (1 + dt L~) rho_n for the walker list, in the
    importance-sampled representation.  If ``non_initiator`` (bool per entry) is
    given, off-diagonal progeny of those parents on configurations that are
    neither occupied nor diagonal is removed (Sec. IV.A)."""
    N = Lx * Ly
    D = 2 ** N
    L = liouvillian(Lx, Ly, Jx, Jy, Jz, gamma, S=S, is_p=is_p, hx=hx, hy=hy).tocsc()
    cols = vec_index(keys, N)
    v = np.asarray(re, float) + 1j * np.asarray(im, float)
    sub = L[:, cols].tocoo()
    data = sub.data.copy()
    if non_initiator is not None:
        occupied = np.zeros(D * D, bool)
        occupied[cols] = True
        child = sub.row
        par = cols[sub.col]
        child_diag = (child % D) == (child // D)
        drop = (np.asarray(non_initiator)[sub.col] & (child != par) & ~occupied[child]
                & ~child_diag)
        data[drop] = 0.0
    mat = sp.coo_matrix((data, (sub.row, sub.col)), shape=(D * D, len(cols))).tocsr()
    out = dt * (mat @ v)
    out[cols] += v
    return out


_H_CACHE = {}


def column(Lx, Ly, Jx, Jy, Jz, gamma, l, m, S=0.0, is_p=0.0, hx=0.0, hy=0.0):
    """One column of the shifted, importance-sampled Liouvillian, for parent
    |l><m|, from the sparse H and the jump matrices (no Kronecker product of the
    full superoperator; usable up to 4x4).  Returns {(ket, bra): value}."""
    N = Lx * Ly
    key = (Lx, Ly, Jx, Jy, Jz, hx, hy)
    if key not in _H_CACHE:
        Hm = hamiltonian(Lx, Ly, Jx, Jy, Jz, hx, hy)
        _H_CACHE[key] = ((Hm.tocsc(), Hm.tocsr()),
                         [F.tocsc() for F in jump_ops(Lx, Ly)])
    (H, Hr), Fs = _H_CACHE[key]
    out = {}

    def add(i, j, v):
        if v != 0:
            out[(i, j)] = out.get((i, j), 0) + v

    # -i H |l><m|  : children |i><m| with -i H_il
    col = H[:, l]
    for i, v in zip(col.indices, col.data):
        add(int(i), m, -1j * v)
    # +i |l><m| H  : children |l><j| with +i H_mj
    row = Hr[m]            # H is Hermitian (not symmetric once the field has sigma^y)
    for j, v in zip(row.indices, row.data):
        add(l, int(j), 1j * v)
    for F in Fs:
        fl = F[:, l]
        fm = F[:, m]
        for i, a in zip(fl.indices, fl.data):
            for j, b in zip(fm.indices, fm.data):
                add(int(i), int(j), gamma * a * np.conj(b))
        FdF = (F.conj().T @ F).tocsc()
        add(l, m, -0.5 * gamma * (FdF[l, l] + FdF[m, m]))
    add(l, m, -S)
    if is_p != 0.0:
        wpar = 1.0 if l == m else np.exp(-is_p)
        for (i, j) in list(out):
            if (i, j) != (l, m):
                wch = 1.0 if i == j else np.exp(-is_p)
                out[(i, j)] *= wch / wpar
    return out
