"""MI355X (gfx950) DDQMC propagation step -- Python side of the C ABI.

``Solve``, ``Batch`` and ``Pool`` wrap the handles of include/ddqmc.h
(ddqmc_create / ddqmc_step / ddqmc_observables / ddqmc_destroy and the batched
and serving calls).  The walker step itself runs in the library's HIP kernels;
this module only marshals arguments.  PyTorch is optional: a ``torch.cuda``
stream can be handed over with ``stream=torch.cuda.current_stream()``.
"""
import ctypes

import numpy as np

from ._lib import (DDQMCError, NO_INITIATOR, NSUM, PER_WALKER, Obs, Params, SERIES_W, SUM_NAMES, check, lib,
                   make_params, ptr)

STAGES = ("scan", "gather", "loud", "heavy", "seal", "histogram", "sort", "count", "merge",
          "finalize")

__all__ = ["Solve", "Batch", "Pool", "make_params", "DDQMCError", "NO_INITIATOR", "PER_WALKER",
           "SUM_NAMES",
           "dev_uniforms", "dev_binom", "dev_binom_noalloc", "dev_math", "dev_quiet",
           "workspace_query", "ratio_se",
           "plan_growth"]


def _stream_ptr(stream):
    if stream is None:
        return None
    s = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(s))


def _obs_dict(o):
    d = {f: getattr(o, f) for f, _ in Obs._fields_ if f not in ("last", "acc")}
    d["last"] = dict(zip(SUM_NAMES, list(o.last)))
    d["acc"] = dict(zip(SUM_NAMES, list(o.acc)))
    return d


class _Handle:
    _h = None

    def _step(self, n):
        check(lib().ddqmc_step(self._h, int(n)), "ddqmc_step")

    def close(self):
        if self._h:
            lib().ddqmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def observables(self, slot=0):
        o = Obs()
        check(lib().ddqmc_slot_observables(self._h, int(slot), ctypes.byref(o)),
              "ddqmc_observables")
        return _obs_dict(o)

    def walkers(self, slot=0):
        n = ctypes.c_int64()
        lib().ddqmc_get_walkers(self._h, int(slot), None, None, None, 0, ctypes.byref(n))
        cap = max(n.value, 1)
        k = np.empty(cap, np.uint64)
        r = np.empty(cap, np.int32)
        i = np.empty(cap, np.int32)
        check(lib().ddqmc_get_walkers(self._h, int(slot), ptr(k, ctypes.c_uint64),
                                      ptr(r, ctypes.c_int32), ptr(i, ctypes.c_int32), cap,
                                      ctypes.byref(n)), "ddqmc_get_walkers")
        return k[:n.value], r[:n.value], i[:n.value]

    def scalars(self, slot=0):
        S = ctypes.c_double()
        mode = ctypes.c_int32()
        step = ctypes.c_int64()
        nwp = ctypes.c_int64()
        check(lib().ddqmc_get_scalars(self._h, int(slot), ctypes.byref(S), ctypes.byref(mode),
                                      ctypes.byref(step), ctypes.byref(nwp)), "get_scalars")
        return dict(S=S.value, mode=mode.value, step=step.value, nw_prev=nwp.value)

    def set_scalars(self, S, mode, step, nw_prev, slot=0):
        check(lib().ddqmc_set_scalars(self._h, int(slot), float(S), int(mode), int(step),
                                      int(nw_prev)), "set_scalars")

    def series(self, slot=0):
        n = ctypes.c_int64()
        check(lib().ddqmc_get_series(self._h, int(slot), None, 0, ctypes.byref(n)), "series")
        rows = np.zeros((n.value, SERIES_W), np.int64)
        check(lib().ddqmc_get_series(self._h, int(slot), ptr(rows, ctypes.c_int64), n.value,
                                     ctypes.byref(n)), "series")
        return rows

    def step_counts(self):
        """(entries in, spawn records, entries out, loud entries, heavy entries)
        for every step so far."""
        n = ctypes.c_int64()
        check(lib().ddqmc_get_step_counts(self._h, None, 0, ctypes.byref(n)), "step_counts")
        rows = np.zeros((n.value, 5), np.int64)
        check(lib().ddqmc_get_step_counts(self._h, ptr(rows, ctypes.c_int64), n.value,
                                          ctypes.byref(n)), "step_counts")
        return rows

    def list_size(self):
        n = ctypes.c_int64()
        check(lib().ddqmc_list_size(self._h, ctypes.byref(n)), "list_size")
        return n.value

    def set_profiling(self, every=1):
        """Stage events on every `every`-th step (True: every step, 0 or False: off)."""
        check(lib().ddqmc_set_profiling(self._h, int(every)), "set_profiling")

    def set_graph_steps(self, k):
        """Run k steps per HIP graph launch (k even, 0 = one launch per kernel)."""
        check(lib().ddqmc_set_graph_steps(self._h, int(k)), "set_graph_steps")

    def set_heavy_fork(self, mode):
        """Large-population entries on a second stream: 0 by list size, 1 always, -1 never."""
        check(lib().ddqmc_set_heavy_fork(self._h, int(mode)), "set_heavy_fork")

    def set_tree_queue(self, places):
        """Member-tree places per loud chunk (0: the most the kernel holds); entries
        whose trees find no room take the general path, with the same results."""
        check(lib().ddqmc_set_tree_queue(self._h, int(places)), "set_tree_queue")

    def set_field_limit(self, spawns):
        """With the field in every solve: entries with this many walkers spawned
        along one element part by one part of their walkers (1..20, default 20)
        go to the general routine; the results are the same either way."""
        check(lib().ddqmc_set_field_limit(self._h, int(spawns)), "set_field_limit")

    def set_loud_grid(self, mode):
        """Loud kernel grid: 0 chosen per chunk of steps, 1 resident blocks, 2 a block
        per chunk of entries (same results either way)."""
        check(lib().ddqmc_set_loud_grid(self._h, int(mode)), "set_loud_grid")

    def set_tiles(self, sort_it, merge_it):
        """Sort tile: sort_it records per thread (4, 8, 16); merge tile: merge_it
        merged positions per thread (4, 8).  Clears a tile table."""
        check(lib().ddqmc_set_tiles(self._h, int(sort_it), int(merge_it)), "set_tiles")

    def set_tile_table(self, rows):
        """rows: [(min_entries, sort_it, merge_it), ...] ascending in min_entries;
        before each chunk of steps the shape of the last row at or below the
        list size is used.  [] clears it."""
        n = len(rows)
        me = np.array([r[0] for r in rows], np.int64)
        si = np.array([r[1] for r in rows], np.int32)
        mi = np.array([r[2] for r in rows], np.int32)
        check(lib().ddqmc_set_tile_table(self._h, n, ptr(me, ctypes.c_int64),
                                         ptr(si, ctypes.c_int32), ptr(mi, ctypes.c_int32)),
              "set_tile_table")

    def tiles(self):
        """(sort_it, merge_it) in use."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(lib().ddqmc_get_tiles(self._h, ctypes.byref(a), ctypes.byref(b)), "get_tiles")
        return a.value, b.value

    def device_bytes(self):
        """(device bytes the handle holds, its list capacity in entries)."""
        n = ctypes.c_size_t()
        cap = ctypes.c_int64()
        check(lib().ddqmc_device_bytes(self._h, ctypes.byref(n), ctypes.byref(cap)),
              "device_bytes")
        return n.value, cap.value

    def set_capacity_limit(self, max_entries):
        """Ceiling on the list and record capacities growth may reach (0: none)."""
        check(lib().ddqmc_set_capacity_limit(self._h, int(max_entries)), "set_capacity_limit")

    def stage_times(self):
        ms = (ctypes.c_double * len(STAGES))()
        steps = ctypes.c_int64()
        check(lib().ddqmc_stage_times(self._h, ms, ctypes.byref(steps)), "stage_times")
        return dict(zip(STAGES, list(ms))), steps.value


class Solve(_Handle):
    """One steady-state solve (ddqmc_create).  With ``workspace`` (a device
    buffer: a torch tensor, or an (address, bytes) pair) the handle lives in
    that memory (ddqmc_create_in), which must stay alive and unmoved until
    close(); its buffers then never grow."""

    def __init__(self, params=None, stream=None, workspace=None, **kw):
        self.params = params if params is not None else make_params(**kw)
        h = ctypes.c_void_p()
        if workspace is None:
            check(lib().ddqmc_create(ctypes.byref(self.params), _stream_ptr(stream),
                                     ctypes.byref(h)), "ddqmc_create")
        else:
            if isinstance(workspace, tuple):
                addr, nbytes = workspace
            else:
                addr = workspace.data_ptr()
                nbytes = workspace.numel() * workspace.element_size()
            self._workspace = workspace  # kept alive with the handle
            check(lib().ddqmc_create_in(ctypes.byref(self.params), ctypes.c_void_p(int(addr)),
                                        int(nbytes), _stream_ptr(stream), ctypes.byref(h)),
                  "ddqmc_create_in")
        self._h = h

    def step(self, n=1):
        self._step(n)

    def set_walkers(self, keys, re, im):
        k = np.ascontiguousarray(keys, np.uint64)
        r = np.ascontiguousarray(re, np.int32)
        i = np.ascontiguousarray(im, np.int32)
        check(lib().ddqmc_set_walkers(self._h, ptr(k, ctypes.c_uint64), ptr(r, ctypes.c_int32),
                                      ptr(i, ctypes.c_int32), len(k)), "ddqmc_set_walkers")

    def get_state(self):
        n = ctypes.c_size_t()
        check(lib().ddqmc_get_state(self._h, None, 0, ctypes.byref(n)), "get_state")
        buf = ctypes.create_string_buffer(n.value)
        check(lib().ddqmc_get_state(self._h, buf, n.value, ctypes.byref(n)), "get_state")
        return buf.raw

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().ddqmc_set_state(self._h, buf, len(blob)), "set_state")


class Batch(_Handle):
    """Independent solves advanced together (ddqmc_batch_create)."""

    def __init__(self, params_list, stream=None):
        arr = (Params * len(params_list))(*params_list)
        h = ctypes.c_void_p()
        check(lib().ddqmc_batch_create(arr, len(params_list), _stream_ptr(stream),
                                       ctypes.byref(h)), "ddqmc_batch_create")
        self._h = h
        self.count = len(params_list)

    def step(self, n=1):
        check(lib().ddqmc_batch_step(self._h, int(n)), "ddqmc_batch_step")


class Pool(_Handle):
    """Continuous batching: solves enter and leave slots between steps."""

    def __init__(self, slots, max_sites, capacity_hint=0, stream=None):
        h = ctypes.c_void_p()
        check(lib().ddqmc_pool_create(int(slots), int(max_sites), int(capacity_hint),
                                      _stream_ptr(stream), ctypes.byref(h)), "ddqmc_pool_create")
        self._h = h
        self.slots = slots

    def admit(self, params):
        s = ctypes.c_int32()
        check(lib().ddqmc_slot_admit(self._h, ctypes.byref(params), ctypes.byref(s)), "admit")
        return s.value

    def retire(self, slot):
        check(lib().ddqmc_slot_retire(self._h, int(slot)), "retire")

    def step(self, n=1):
        self._step(n)


def workspace_query(params, capacity=0):
    n = ctypes.c_size_t()
    check(lib().ddqmc_workspace_query(ctypes.byref(params), int(capacity), ctypes.byref(n)),
          "workspace_query")
    return n.value


def plan_growth(cap_main, cap_sp, need_main, seg_need, key_bytes, free_bytes, total_bytes,
                cap_limit=0):
    """The library's buffer-growth arithmetic (host only): returns (code, new list
    capacity, new record capacity, bytes of the new list and scratch arena)."""
    nm, ns, nb = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().ddqmc_plan_growth(int(cap_main), int(cap_sp), int(need_main), int(seg_need),
                                 int(key_bytes), int(free_bytes), int(total_bytes),
                                 int(cap_limit), ctypes.byref(nm), ctypes.byref(ns),
                                 ctypes.byref(nb))
    return rc, nm.value, ns.value, nb.value


def ratio_se(num, den):
    """The library's blocking / delta-method error of mean(num) / mean(den) (host)."""
    a = np.ascontiguousarray(num, np.float64)
    b = np.ascontiguousarray(den, np.float64)
    if a.shape != b.shape or a.ndim != 1:
        raise ValueError("ratio_se: num and den must be 1-d series of one length")
    se = ctypes.c_double()
    check(lib().ddqmc_ratio_se(ptr(a, ctypes.c_double), ptr(b, ctypes.c_double), len(a),
                               ctypes.byref(se)), "ratio_se")
    return se.value


def dev_uniforms(seed, solve_id, cfg, step, draw, count):
    out = np.zeros(count, np.float64)
    check(lib().ddqmc_dev_uniforms(seed, solve_id, cfg, step, draw, count,
                                   ptr(out, ctypes.c_double)), "dev_uniforms")
    return out


def dev_binom(n, p, mode, seed, count):
    out = np.zeros(count, np.int64)
    check(lib().ddqmc_dev_binom(int(n), float(p), int(mode), int(seed), int(count),
                                ptr(out, ctypes.c_int64)), "dev_binom")
    return out


def dev_binom_noalloc(n, p, mode, seed, count):
    """dev_binom through the entry point that allocates no device memory (its
    samples are staged in the library's static scratch; count <= 2^20)."""
    out = np.zeros(count, np.int64)
    check(lib().ddqmc_dev_binom_noalloc(int(n), float(p), int(mode), int(seed), int(count),
                                        ptr(out, ctypes.c_int64)), "dev_binom_noalloc")
    return out


def dev_quiet(p, n, u):
    """The spawn scan's quiet test on given inputs: p (count, 4) channel
    probabilities, n (count, 2) walker counts |R|, |I|, u (count,) primary
    uniforms.  Returns int32 (count,): bit 0 quiet, bit 1 decided by the
    single-precision estimate."""
    p = np.ascontiguousarray(p, np.float64).reshape(-1, 4)
    n = np.ascontiguousarray(n, np.int64).reshape(-1, 2)
    u = np.ascontiguousarray(u, np.float64).ravel()
    if not (len(p) == len(n) == len(u)):
        raise ValueError("dev_quiet: p, n and u must describe the same number of entries")
    out = np.zeros(len(u), np.int32)
    check(lib().ddqmc_dev_quiet(ptr(p, ctypes.c_double), ptr(n, ctypes.c_int64),
                                ptr(u, ctypes.c_double), len(u), ptr(out, ctypes.c_int32)),
          "dev_quiet")
    return out


def dev_math(x):
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(4 * len(x), np.float64)
    check(lib().ddqmc_dev_math(ptr(x, ctypes.c_double), len(x), ptr(out, ctypes.c_double)),
          "dev_math")
    return out.reshape(-1, 4)
