"""Host drivers for many solves on one GPU: a batch of replicas stepped together,
and a serving loop with continuous batching.

Both run every step through the library's kernels (one launch per stage for
all solves of the handle); this module only decides
which solve sits in which slot and when a solve is done.

Serving loop (``serve``): requests arrive over time; a request is admitted into
a free slot of a ``Pool`` while the pool's list (all solves' occupied entries,
which sets its device-memory footprint) is below an entry budget; the pool
advances in ticks of ``tick`` steps; after each tick a
solve whose magnetisation M_z has a standard error below ``se_target`` (with
at least ``min_accum`` accumulated steps after its equilibration), that has run
``max_steps`` steps, or whose list has grown past ``max_entries`` (a per-request
memory limit) leaves its slot.  The standard error is the library's
blocking / delta-method error of the ratio estimator (Sec. III.A, V.A).
"""
import time
from collections import deque

import numpy as np

from . import Batch, Pool, Solve, make_params
from ._lib import ESTATE, DDQMCError


def _done(obs, se_target, min_accum, max_steps, max_entries):
    """(finished, converged, over the memory limit) for a solve with observables obs."""
    converged = (obs["n_accum"] >= min_accum and np.isfinite(obs["se_mz"])
                 and obs["se_mz"] < se_target)
    over = obs["last"]["n_entries"] > max_entries
    return converged or over or obs["step"] >= max_steps, converged, over


def serve(requests, slots=64, max_sites=16, entry_budget=60_000_000, tick=50,
          se_target=1e-3, min_accum=512, max_steps=2000, max_entries=4_000_000, graph_k=0,
          stream=None, log=None):
    """Run the request stream through one pool.

    requests: list of dicts with "arrival" (seconds from the start) and "params"
    (keyword arguments of make_params).  Returns one record per request:
    arrival, admitted, finished (seconds), steps, converged, mz, se_mz.
    """
    order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival"])
    pending = deque(order)
    queue = deque()
    pool = Pool(slots, max_sites, stream=stream)
    if graph_k:
        pool.set_graph_steps(graph_k)
    active = {}  # slot -> request index
    out = [None] * len(requests)
    t0 = time.perf_counter()
    ticks = 0
    while pending or queue or active:
        now = time.perf_counter() - t0
        while pending and requests[pending[0]]["arrival"] <= now:
            queue.append(pending.popleft())
        # admission by footprint, in arrival order
        entries = pool.list_size() if active else 0
        while queue and len(active) < slots and entries < entry_budget:
            i = queue[0]
            try:
                s = pool.admit(make_params(**requests[i]["params"]))
            except DDQMCError as e:
                if e.code != ESTATE:
                    raise
                break  # every free slot is still being vacated: after the next tick
            queue.popleft()
            active[s] = i
            out[i] = dict(arrival=requests[i]["arrival"], admitted=now)
        if not active:
            if pending:  # idle until the next arrival
                time.sleep(max(0.0, requests[pending[0]]["arrival"] - now))
            continue
        pool.step(tick)
        ticks += 1
        now = time.perf_counter() - t0
        for s in list(active):
            i = active[s]
            obs = pool.observables(s)
            fin, conv, over = _done(obs, se_target, min_accum, max_steps, max_entries)
            if fin:
                pool.retire(s)
                del active[s]
                out[i].update(finished=now, steps=int(obs["step"]), converged=bool(conv),
                              over_limit=bool(over), entries=int(obs["last"]["n_entries"]),
                              mz=float(obs["mz"]), se_mz=float(obs["se_mz"]))
                if log:
                    log(f"request {i} done at {now:.2f}s after {obs['step']} steps, "
                        f"{obs['last']['n_entries']} entries (converged={conv}, over={over}, "
                        f"{len(active)} active, {len(queue)} queued)")
    pool.close()
    return out, ticks


def solve_alone(params, steps, tick=50, graph_k=0, stream=None):
    """One request on its own handle, stepped in ticks of ``tick`` for exactly
    ``steps`` steps (the count the pool took, so the list and the observables
    are the pool's).  Returns (seconds, observables)."""
    g = Solve(make_params(**params), stream=stream)
    if graph_k:
        g.set_graph_steps(graph_k)
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(tick, steps - done)
        g.step(n)
        g.observables()  # the per-tick check the serving loop makes
        done += n
    dt = time.perf_counter() - t0
    obs = g.observables()
    g.close()
    return dt, obs


def replicas_batched(cfgs, steps, graph_k=0, stream=None):
    """All replicas in one batch handle: (seconds, list of observables)."""
    b = Batch([make_params(**c) for c in cfgs], stream=stream)
    if graph_k:
        b.set_graph_steps(graph_k)
    b.step(1)  # buffers sized, graphs not yet captured: excluded from the timing
    t0 = time.perf_counter()
    b.step(steps - 1)
    b.observables(0)
    dt = time.perf_counter() - t0
    obs = [b.observables(i) for i in range(len(cfgs))]
    lists = [b.walkers(i) for i in range(len(cfgs))]
    b.close()
    return dt, obs, lists


def replicas_sequential(cfgs, steps, graph_k=0, stream=None, keep_lists=True, log=None):
    """The same replicas one after another, each on its own handle."""
    total = 0.0
    obs, lists = [], []
    for r, c in enumerate(cfgs):
        g = Solve(make_params(**c), stream=stream)
        if graph_k:
            g.set_graph_steps(graph_k)
        g.step(1)
        t0 = time.perf_counter()
        g.step(steps - 1)
        g.observables()
        total += time.perf_counter() - t0
        obs.append(g.observables())
        if keep_lists:
            lists.append(g.walkers())
        g.close()
        if log:
            log(f"replica {r} alone: {total:.2f} s so far")
    return total, obs, lists
