"""ctypes binding of ``libddqmc.so`` (the C ABI in include/ddqmc.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddqmc.so")

OK, EINVAL, ENOMEM, ECAPACITY, EOVERFLOW, EEXTINCT, EHIP, ESTATE, ERNG = 0, -1, -2, -3, -4, -5, \
    -6, -7, -8
NO_INITIATOR = 1
PER_WALKER = 2  # walker-by-walker sampling (Sec. II), the per-entry scheme's ablation
SUM_NAMES = ("t_re", "t_im", "n_w", "z", "x", "y", "cxx", "cyy", "czz", "w_tot", "n_entries")
NSUM = len(SUM_NAMES)
SERIES_W = 3 + NSUM


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
        ("Jx", ctypes.c_double), ("Jy", ctypes.c_double), ("Jz", ctypes.c_double),
        ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
        ("n_a", ctypes.c_int32),
        ("target_walkers", ctypes.c_int64), ("initial_walkers", ctypes.c_int64),
        ("is_p", ctypes.c_double), ("shift_damping", ctypes.c_double),
        ("shift_init", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("solve_id", ctypes.c_uint32),
        ("n_equil", ctypes.c_int64), ("capacity_hint", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
        ("hx", ctypes.c_double), ("hy", ctypes.c_double),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("shift", ctypes.c_double),
        ("mode", ctypes.c_int32), ("status", ctypes.c_int32),
        ("last", ctypes.c_int64 * NSUM), ("n_accum", ctypes.c_int64),
        ("acc", ctypes.c_int64 * NSUM),
        ("mx", ctypes.c_double), ("my", ctypes.c_double), ("mz", ctypes.c_double),
        ("cxx", ctypes.c_double), ("cyy", ctypes.c_double), ("czz", ctypes.c_double),
        ("se_mx", ctypes.c_double), ("se_my", ctypes.c_double), ("se_mz", ctypes.c_double),
        ("se_cxx", ctypes.c_double), ("se_cyy", ctypes.c_double), ("se_czz", ctypes.c_double),
    ]


DEFAULTS = dict(Lx=2, Ly=2, Jx=0.9, Jy=1.0, Jz=1.0, gamma=1.0, dt=0.01, n_a=3,
                target_walkers=1000, initial_walkers=100, is_p=0.0, shift_damping=0.05,
                shift_init=-0.5, seed=0, solve_id=0, n_equil=0, capacity_hint=0, flags=0,
                hx=0.0, hy=0.0)


def make_params(**kw):
    d = dict(DEFAULTS)
    for k in kw:
        if k not in d:
            raise KeyError(k)
    d.update(kw)
    p = Params(**d)
    p.struct_size = ctypes.sizeof(Params)
    return p


_P = ctypes.POINTER
_vp = ctypes.c_void_p
# name -> (restype, argtypes); the names are those of include/ddqmc.h
SIGNATURES = {
    "ddqmc_create": (ctypes.c_int, [_P(Params), _vp, _P(_vp)]),
    "ddqmc_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "ddqmc_observables": (ctypes.c_int, [_vp, _P(Obs)]),
    "ddqmc_destroy": (ctypes.c_int, [_vp]),
    "ddqmc_batch_create": (ctypes.c_int, [_P(Params), ctypes.c_int32, _vp, _P(_vp)]),
    "ddqmc_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "ddqmc_batch_observables": (ctypes.c_int, [_vp, ctypes.c_int32, _P(Obs)]),
    "ddqmc_pool_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _vp,
                                         _P(_vp)]),
    "ddqmc_slot_admit": (ctypes.c_int, [_vp, _P(Params), _P(ctypes.c_int32)]),
    "ddqmc_slot_retire": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_slot_observables": (ctypes.c_int, [_vp, ctypes.c_int32, _P(Obs)]),
    "ddqmc_list_size": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "ddqmc_get_walkers": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_uint64),
                                         _P(ctypes.c_int32), _P(ctypes.c_int32), ctypes.c_int64,
                                         _P(ctypes.c_int64)]),
    "ddqmc_set_walkers": (ctypes.c_int, [_vp, _P(ctypes.c_uint64), _P(ctypes.c_int32),
                                         _P(ctypes.c_int32), ctypes.c_int64]),
    "ddqmc_get_scalars": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_double),
                                         _P(ctypes.c_int32), _P(ctypes.c_int64),
                                         _P(ctypes.c_int64)]),
    "ddqmc_set_scalars": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int64]),
    "ddqmc_get_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _P(ctypes.c_size_t)]),
    "ddqmc_set_state": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "ddqmc_get_series": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64), ctypes.c_int64,
                                        _P(ctypes.c_int64)]),
    "ddqmc_get_step_counts": (ctypes.c_int, [_vp, _P(ctypes.c_int64), ctypes.c_int64,
                                             _P(ctypes.c_int64)]),
    "ddqmc_workspace_query": (ctypes.c_int, [_P(Params), ctypes.c_int64, _P(ctypes.c_size_t)]),
    "ddqmc_create_in": (ctypes.c_int, [_P(Params), _vp, ctypes.c_size_t, _vp, _P(_vp)]),
    "ddqmc_device_bytes": (ctypes.c_int, [_vp, _P(ctypes.c_size_t), _P(ctypes.c_int64)]),
    "ddqmc_set_capacity_limit": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "ddqmc_ratio_se": (ctypes.c_int, [_P(ctypes.c_double), _P(ctypes.c_double), ctypes.c_int64,
                                      _P(ctypes.c_double)]),
    "ddqmc_plan_growth": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_uint64, _P(ctypes.c_uint64),
                                         _P(ctypes.c_uint64), _P(ctypes.c_uint64)]),
    "ddqmc_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_set_graph_steps": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_set_heavy_fork": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_set_tree_queue": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_set_field_limit": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_set_loud_grid": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "ddqmc_stage_times": (ctypes.c_int, [_vp, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "ddqmc_set_tiles": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "ddqmc_set_tile_table": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64),
                                            _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "ddqmc_get_tiles": (ctypes.c_int, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    "ddqmc_dev_uniforms": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                          _P(ctypes.c_double)]),
    "ddqmc_dev_binom": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_int64, _P(ctypes.c_int64)]),
    "ddqmc_dev_math": (ctypes.c_int, [_P(ctypes.c_double), ctypes.c_int64, _P(ctypes.c_double)]),
    "ddqmc_dev_binom_noalloc": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                               ctypes.c_uint64, ctypes.c_int64,
                                               _P(ctypes.c_int64)]),
    "ddqmc_dev_quiet": (ctypes.c_int, [_P(ctypes.c_double), _P(ctypes.c_int64), _P(ctypes.c_double),
                                       ctypes.c_int64, _P(ctypes.c_int32)]),
    "ddqmc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def lib():
    """Load libddqmc.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DDQMCError(RuntimeError):
    def __init__(self, code, what):
        msg = lib().ddqmc_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def check(rc, what):
    if rc != OK:
        raise DDQMCError(rc, what)
    return rc


def ptr(a, ct):
    return a.ctypes.data_as(_P(ct))
