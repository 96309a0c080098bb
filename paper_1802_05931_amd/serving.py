"""Host drivers for many solves on one GPU: a batch of replicas stepped together,
and a serving loop with continuous batching.

Both run every step through the library's kernels (one launch per stage for
all solves of the handle); this module only decides
which solve sits in which slot and when a solve is done.

Serving loop (``serve``): requests arrive over time; a request is admitted, in
arrival order, into a free slot of a ``Pool`` while the device bytes projected
for the admitted solves stay within ``hbm_budget``.  A request's projection is
the library's exact workspace size (ddqmc_workspace_query) for the largest list
it may hold: its lattice's reachable configurations (the even-parity half of
the 4^N density-matrix configurations, all of them with the in-plane field),
at most the per-request entry limit ``max_entries``.  The pool advances in ticks of ``tick`` steps; after each tick a
solve whose magnetisation M_z has a standard error below ``se_target`` (with
at least ``min_accum`` accumulated steps after its equilibration), that has run
``max_steps`` steps, or whose list has grown past ``max_entries`` leaves its
slot.  If a tick fails because the pool's buffers cannot grow (device memory
or the largest buffer), the pool is at its last completed step: the solve
with the largest list is evicted and the tick is run again.  The standard
error is the library's blocking / delta-method error of the ratio estimator
(Sec. III.A, V.A).
"""
import time
from collections import deque

import numpy as np

from . import Batch, Pool, Solve, make_params, workspace_query
from ._lib import ECAPACITY, ENOMEM, ESTATE, DDQMCError


def projected_bytes(params, max_entries):
    """Device bytes a request may come to hold: the workspace of a one-slot
    handle whose list capacity is the smaller of the lattice's reachable
    configurations (popcount(ket) + popcount(bra) even: 2^(2N-1); with the
    in-plane field, which breaks that parity, all 4^N) and the per-request
    entry limit."""
    n = int(params["Lx"]) * int(params["Ly"])
    field = params.get("hx", 0.0) != 0.0 or params.get("hy", 0.0) != 0.0
    cap = min(1 << (2 * n if field else 2 * n - 1), int(max_entries))
    return workspace_query(make_params(**params), cap)


def _done(obs, se_target, min_accum, max_steps, max_entries):
    """(finished, converged, over the memory limit) for a solve with observables obs."""
    converged = (obs["n_accum"] >= min_accum and np.isfinite(obs["se_mz"])
                 and obs["se_mz"] < se_target)
    over = obs["last"]["n_entries"] > max_entries
    return converged or over or obs["step"] >= max_steps, converged, over


def serve(requests, slots=64, max_sites=16, hbm_budget=32 << 30, tick=50,
          se_target=1e-3, min_accum=512, max_steps=2000, max_entries=4_000_000, graph_k=0,
          stream=None, log=None, clock=None, sleep=None):
    """Run the request stream through one pool.

    requests: list of dicts with "arrival" (seconds from the start) and "params"
    (keyword arguments of make_params).  ``clock`` (seconds since the start)
    and ``sleep`` default to the wall clock; a test replays arrivals with its
    own.  Returns (one record per request: arrival, admitted, finished
    (seconds), steps, converged, over_limit, evicted, entries, mz, se_mz;
    stats: ticks, the most solves and projected bytes held at once,
    evictions)."""
    if clock is None:
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
    if sleep is None:
        sleep = time.sleep
    order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival"])
    proj = {i: projected_bytes(requests[i]["params"], max_entries) for i in order}
    pending = deque(order)
    queue = deque()
    pool = Pool(slots, max_sites, stream=stream)
    if graph_k:
        pool.set_graph_steps(graph_k)
    active = {}  # slot -> request index
    held = 0     # projected bytes of the active solves
    out = [None] * len(requests)
    stats = dict(ticks=0, max_active=0, max_projected_bytes=0, evicted=0, admission_order=[])

    def finish(s, now, evicted=False):
        nonlocal held
        i = active.pop(s)
        held -= proj[i]
        obs = pool.observables(s)
        fin, conv, over = _done(obs, se_target, min_accum, max_steps, max_entries)
        pool.retire(s)
        out[i].update(finished=now, steps=int(obs["step"]), converged=bool(conv and not evicted),
                      over_limit=bool(over), evicted=bool(evicted),
                      entries=int(obs["last"]["n_entries"]), mz=float(obs["mz"]),
                      se_mz=float(obs["se_mz"]))
        if log:
            log(f"request {i} {'evicted' if evicted else 'done'} at {now:.2f}s after "
                f"{obs['step']} steps, {obs['last']['n_entries']} entries (converged={conv}, "
                f"over={over}, {len(active)} active, {len(queue)} queued)")

    while pending or queue or active:
        now = clock()
        while pending and requests[pending[0]]["arrival"] <= now:
            queue.append(pending.popleft())
        # admission in arrival order while the projected bytes fit (a request
        # larger than the whole budget runs once the pool is empty)
        while queue and len(active) < slots:
            i = queue[0]
            if active and held + proj[i] > hbm_budget:
                break
            try:
                s = pool.admit(make_params(**requests[i]["params"]))
            except DDQMCError as e:
                if e.code != ESTATE:
                    raise
                break  # every free slot is still being vacated: after the next tick
            queue.popleft()
            active[s] = i
            held += proj[i]
            out[i] = dict(arrival=requests[i]["arrival"], admitted=now)
            stats["admission_order"].append(i)
        stats["max_active"] = max(stats["max_active"], len(active))
        stats["max_projected_bytes"] = max(stats["max_projected_bytes"], held)
        if not active:
            if pending:  # idle until the next arrival
                sleep(max(0.0, requests[pending[0]]["arrival"] - now))
            continue
        try:
            pool.step(tick)
        except DDQMCError as e:
            if e.code not in (ENOMEM, ECAPACITY):
                raise
            # the pool's buffers could not grow; it is at its last completed
            # step: the largest solve leaves, and the tick runs again
            big = max(active, key=lambda s: pool.observables(s)["last"]["n_entries"])
            finish(big, clock(), evicted=True)
            stats["evicted"] += 1
            continue
        stats["ticks"] += 1
        now = clock()
        for s in list(active):
            fin, _, _ = _done(pool.observables(s), se_target, min_accum, max_steps, max_entries)
            if fin:
                finish(s, now)
    pool.close()
    return out, stats


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


def replicas_batched(cfgs, steps, graph_k=0, stream=None, tile_rows=None):
    """All replicas in one batch handle: (seconds, list of observables).
    tile_rows: a tuned tile table (rows (min_entries, sort_it, merge_it))."""
    b = Batch([make_params(**c) for c in cfgs], stream=stream)
    if graph_k:
        b.set_graph_steps(graph_k)
    if tile_rows:
        b.set_tile_table([tuple(r) for r in tile_rows])
    b.step(1)  # buffers sized, graphs not yet captured: excluded from the timing
    t0 = time.perf_counter()
    b.step(steps - 1)
    b.observables(0)
    dt = time.perf_counter() - t0
    obs = [b.observables(i) for i in range(len(cfgs))]
    lists = [b.walkers(i) for i in range(len(cfgs))]
    b.close()
    return dt, obs, lists


def replicas_sequential(cfgs, steps, graph_k=0, stream=None, keep_lists=True, log=None,
                        tile_rows=None):
    """The same replicas one after another, each on its own handle."""
    total = 0.0
    obs, lists = [], []
    for r, c in enumerate(cfgs):
        g = Solve(make_params(**c), stream=stream)
        if graph_k:
            g.set_graph_steps(graph_k)
        if tile_rows:
            g.set_tile_table([tuple(r) for r in tile_rows])
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
