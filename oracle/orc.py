"""ctypes binding of the C oracle (``oracle/ddqmc_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  ``build()`` compiles the C
file with gcc, ``-O2 -ffp-contract=off``, single-threaded, into
``oracle/liborc.so``.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ddqmc_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EEXTINCT, ERNG = 0, -1, -2, -4, -5, -8
NO_INITIATOR = 1
PER_WALKER = 2
SUM_NAMES = ("t_re", "t_im", "n_w", "z", "x", "y", "cxx", "cyy", "czz", "w_tot", "n_entries")
NSUM = len(SUM_NAMES)
SERIES_W = 3 + NSUM


def build(force=True):
    """Compile the oracle with gcc (plain C99, one thread, no FMA contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                           "-Wall", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("Jx", ctypes.c_double), ("Jy", ctypes.c_double), ("Jz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
        ("n_a", ctypes.c_int32),
        ("target_walkers", ctypes.c_int64), ("initial_walkers", ctypes.c_int64),
        ("is_p", ctypes.c_double), ("shift_damping", ctypes.c_double),
        ("shift_init", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("solve_id", ctypes.c_uint32),
        ("n_equil", ctypes.c_int64), ("flags", ctypes.c_uint32),
        ("hx", ctypes.c_double), ("hy", ctypes.c_double),
    ]


DEFAULTS = dict(Lx=2, Ly=2, Jx=0.9, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.01, n_a=3,
                target_walkers=1000, initial_walkers=100, is_p=0.0, shift_damping=0.05,
                shift_init=-0.5, seed=0, solve_id=0, n_equil=0, flags=0, hx=0.0, hy=0.0)


def make_params(**kw):
    d = dict(DEFAULTS)
    for k in kw:
        if k not in d:
            raise KeyError(k)
    d.update(kw)
    return Params(**d)


_lib = None
_P = ctypes.POINTER


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    L = ctypes.CDLL(LIB)
    i64p, i32p, u64p, u32p, dp = (_P(ctypes.c_int64), _P(ctypes.c_int32), _P(ctypes.c_uint64),
                                  _P(ctypes.c_uint32), _P(ctypes.c_double))
    vp = ctypes.c_void_p
    sig = {
        "orc_create": (ctypes.c_int, [_P(Params), _P(vp)]),
        "orc_destroy": (None, [vp]),
        "orc_step": (ctypes.c_int, [vp, ctypes.c_int64]),
        "orc_size": (ctypes.c_int64, [vp]),
        "orc_get_list": (ctypes.c_int, [vp, u64p, i32p, i32p, ctypes.c_int64]),
        "orc_set_list": (ctypes.c_int, [vp, u64p, i32p, i32p, ctypes.c_int64]),
        "orc_get_scalars": (ctypes.c_int, [vp, dp, i32p, i64p, i64p]),
        "orc_set_scalars": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.c_int64]),
        "orc_get_last": (ctypes.c_int, [vp, i64p]),
        "orc_get_acc": (ctypes.c_int, [vp, i64p, i64p]),
        "orc_series_len": (ctypes.c_int64, [vp]),
        "orc_get_series": (ctypes.c_int, [vp, i64p, ctypes.c_int64]),
        "orc_annihilate": (ctypes.c_int, [u64p, i64p, i64p, ctypes.c_int64, u64p, i64p, i64p,
                                          ctypes.c_int64, u64p, i64p, i64p, i64p]),
        "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
        "orc_det_log": (ctypes.c_double, [ctypes.c_double]),
        "orc_det_exp": (ctypes.c_double, [ctypes.c_double]),
        "orc_uniforms": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_int64, dp]),
        "orc_binom_many": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_int64, i64p]),
        "orc_channels_many": (ctypes.c_int, [dp, i64p, ctypes.c_uint64, ctypes.c_int64, i64p]),
        "orc_no_event_prob": (ctypes.c_double, [dp, i64p]),
        "orc_bonds": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, i32p, i32p]),
        "orc_split_many": (ctypes.c_int, [_P(Params), ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_int64, ctypes.c_int64, i64p]),
        "orc_connections": (ctypes.c_int, [_P(Params), ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_double, u64p, u64p, dp, dp, ctypes.c_int32,
                                           dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a, ct):
    return a.ctypes.data_as(_P(ct))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


class Oracle:
    """One DDQMC solve on the CPU, advanced step by step."""

    def __init__(self, params=None, **kw):
        self.params = params if params is not None else make_params(**kw)
        self._h = ctypes.c_void_p()
        _check(lib().orc_create(ctypes.byref(self.params), ctypes.byref(self._h)), "create")
        self.N = self.params.Lx * self.params.Ly

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().orc_step(self._h, int(n)), "step")

    def size(self):
        return int(lib().orc_size(self._h))

    def get_list(self):
        n = self.size()
        k = np.empty(n, np.uint64)
        r = np.empty(n, np.int32)
        i = np.empty(n, np.int32)
        _check(lib().orc_get_list(self._h, _ptr(k, ctypes.c_uint64), _ptr(r, ctypes.c_int32),
                                  _ptr(i, ctypes.c_int32), n), "get_list")
        return k, r, i

    def set_list(self, keys, re, im):
        k = np.ascontiguousarray(keys, np.uint64)
        r = np.ascontiguousarray(re, np.int32)
        i = np.ascontiguousarray(im, np.int32)
        _check(lib().orc_set_list(self._h, _ptr(k, ctypes.c_uint64), _ptr(r, ctypes.c_int32),
                                  _ptr(i, ctypes.c_int32), len(k)), "set_list")

    def scalars(self):
        S = ctypes.c_double()
        mode = ctypes.c_int32()
        step = ctypes.c_int64()
        nwp = ctypes.c_int64()
        lib().orc_get_scalars(self._h, ctypes.byref(S), ctypes.byref(mode), ctypes.byref(step),
                              ctypes.byref(nwp))
        return dict(S=S.value, mode=mode.value, step=step.value, nw_prev=nwp.value)

    def set_scalars(self, S, mode, step, nw_prev):
        lib().orc_set_scalars(self._h, float(S), int(mode), int(step), int(nw_prev))

    def last(self):
        out = np.zeros(NSUM, np.int64)
        lib().orc_get_last(self._h, _ptr(out, ctypes.c_int64))
        return dict(zip(SUM_NAMES, out.tolist()))

    def acc(self):
        out = np.zeros(NSUM, np.int64)
        n = ctypes.c_int64()
        lib().orc_get_acc(self._h, _ptr(out, ctypes.c_int64), ctypes.byref(n))
        return out, n.value

    def series(self):
        n = int(lib().orc_series_len(self._h))
        rows = np.zeros((n, SERIES_W), np.int64)
        _check(lib().orc_get_series(self._h, _ptr(rows, ctypes.c_int64), n), "series")
        return rows


# ---- pieces used by the pin tests -------------------------------------------

def annihilate(ckeys, cre, cim, keys, pr, pi):
    """The step's annihilation on given contributions and list values: the new
    (keys, re, im), int64 values."""
    ck = np.ascontiguousarray(ckeys, np.uint64)
    cr = np.ascontiguousarray(cre, np.int64)
    ci = np.ascontiguousarray(cim, np.int64)
    k = np.ascontiguousarray(keys, np.uint64)
    r = np.ascontiguousarray(pr, np.int64)
    i = np.ascontiguousarray(pi, np.int64)
    cap = max(1, len(k) + len(ck))
    nk = np.empty(cap, np.uint64)
    nr = np.empty(cap, np.int64)
    ni = np.empty(cap, np.int64)
    nout = ctypes.c_int64(0)
    _check(lib().orc_annihilate(_ptr(ck, ctypes.c_uint64), _ptr(cr, ctypes.c_int64),
                                _ptr(ci, ctypes.c_int64), len(ck), _ptr(k, ctypes.c_uint64),
                                _ptr(r, ctypes.c_int64), _ptr(i, ctypes.c_int64), len(k),
                                _ptr(nk, ctypes.c_uint64), _ptr(nr, ctypes.c_int64),
                                _ptr(ni, ctypes.c_int64), ctypes.byref(nout)), "annihilate")
    n = nout.value
    return nk[:n].copy(), nr[:n].copy(), ni[:n].copy()


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32).copy()
    k = np.asarray(key, np.uint32).copy()
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return out


def det_log(x):
    return lib().orc_det_log(float(x))


def det_exp(x):
    return lib().orc_det_exp(float(x))


def uniforms(seed, solve_id, cfg, step, draw, count):
    out = np.zeros(count, np.float64)
    lib().orc_uniforms(seed, solve_id, cfg, step, draw, count, _ptr(out, ctypes.c_double))
    return out


def binom_many(n, p, mode, seed, count):
    out = np.zeros(count, np.int64)
    _check(lib().orc_binom_many(int(n), float(p), int(mode), int(seed), int(count),
                                _ptr(out, ctypes.c_int64)), "binom_many")
    return out


def no_event_prob(p, n):
    """prod_k (1 - p_k)^n_k over the eight channels, in fp64 (Sec. III.B)."""
    pa = np.ascontiguousarray(p, np.float64)
    na = np.ascontiguousarray(n, np.int64)
    if pa.shape != (8,) or na.shape != (8,):
        raise ValueError("no_event_prob: p and n must hold eight channels")
    return float(lib().orc_no_event_prob(_ptr(pa, ctypes.c_double), _ptr(na, ctypes.c_int64)))


def channels_many(p, n, seed, count):
    pa = np.ascontiguousarray(p, np.float64)
    na = np.ascontiguousarray(n, np.int64)
    out = np.zeros((count, 8), np.int64)
    _check(lib().orc_channels_many(_ptr(pa, ctypes.c_double), _ptr(na, ctypes.c_int64), int(seed),
                                   int(count), _ptr(out, ctypes.c_int64)), "channels_many")
    return out


def split_many(params, key, channel, X, count):
    """X walkers of spawning channel `channel` (3/7 jumps, 4/8 hops) of the entry
    `key` placed over its connections by the step's code, count times: rows of N
    counts by site (jumps) or 2 nb counts, ket bonds then bra bonds (hops)."""
    N = params.Lx * params.Ly
    width = N if channel in (3, 7) else 2 * len(bonds(params.Lx, params.Ly))
    out = np.zeros((count, width), np.int64)
    rc = lib().orc_split_many(ctypes.byref(params), int(key), int(channel), int(X), int(count),
                              _ptr(out, ctypes.c_int64))
    if rc < 0:
        raise OracleError(rc, "split_many")
    assert rc == width
    return out


def bonds(Lx, Ly):
    s1 = np.zeros(128, np.int32)
    s2 = np.zeros(128, np.int32)
    nb = lib().orc_bonds(Lx, Ly, _ptr(s1, ctypes.c_int32), _ptr(s2, ctypes.c_int32))
    if nb < 0:
        raise OracleError(nb, "bonds")
    return list(zip(s1[:nb].tolist(), s2[:nb].tolist()))


def connections(params, ket, bra, S=0.0, cap=512):
    ck = np.zeros(cap, np.uint64)
    cb = np.zeros(cap, np.uint64)
    re = np.zeros(cap, np.float64)
    im = np.zeros(cap, np.float64)
    dr = ctypes.c_double()
    di = ctypes.c_double()
    n = lib().orc_connections(ctypes.byref(params), int(ket), int(bra), float(S),
                              _ptr(ck, ctypes.c_uint64), _ptr(cb, ctypes.c_uint64),
                              _ptr(re, ctypes.c_double), _ptr(im, ctypes.c_double), cap,
                              ctypes.byref(dr), ctypes.byref(di))
    if n < 0:
        raise OracleError(n, "connections")
    return ck[:n], cb[:n], re[:n], im[:n], dr.value, di.value


def ratios(acc, N, nb, is_p=0.0):
    """Estimator ratios from accumulated integer sums (Sec. III.A: numerator and
    denominator averaged separately; Sec. IV.B: off-diagonal numerators carry the
    weight e^{p})."""
    s = dict(zip(SUM_NAMES, [int(v) for v in acc]))
    wup = det_exp(is_p)
    den = float(s["t_re"])
    out = {}
    out["mz"] = float(s["z"]) / (float(N) * den)
    out["mx"] = (float(s["x"]) * wup) / (float(N) * den)
    out["my"] = (float(s["y"]) * wup) / (float(N) * den)
    out["cxx"] = (float(s["cxx"]) * wup) / (float(nb) * den)
    out["cyy"] = (float(s["cyy"]) * wup) / (float(nb) * den)
    out["czz"] = float(s["czz"]) / (float(nb) * den)
    return out
