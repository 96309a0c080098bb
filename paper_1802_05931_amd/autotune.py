"""Tuner of the annihilation stage's tile shapes (radix-sort tile and merge-path
tile, ddqmc_set_tiles) per key width and list size.

A workload (one solve or a batch) is stepped to its list of interest; then the
candidate shapes take turns, each for a few steps at a time over several rounds,
with stage events on every step, and the shape with the least sort + merge time
per step wins.  The walker lists do not depend on the shape (the random streams
are keyed on configurations, and the sort and merge are exact), so every shape
sees the same list; the tuner checks that the list is unchanged by comparing
the steps' entry counts with a run of the default shape.  Results go to a JSON
table (``tuned_tiles.json`` next to this file) with one row per tuned list size
and key width; ``apply`` hands a handle the rows for its key width, and the
handle then picks the row for its current list size before each chunk of steps
(ddqmc_set_tile_table).
"""
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_tiles.json")
SHAPES = [(s, m) for s in (4, 8, 16) for m in (4, 8)]
ANNIHILATION_STAGES = ("sort", "count", "merge")


def key_bytes(max_sites, slots=1):
    """Width of the handle's sort key: 2 N configuration bits plus the slot bits."""
    bits = 2 * int(max_sites) + (max(int(slots) - 1, 0)).bit_length()
    return 8 if bits > 32 else 4


def time_shapes(handle, shapes=SHAPES, steps=20, rounds=3):
    """Median sort + merge milliseconds per step of each shape on the handle's
    current workload (the handle keeps stepping: shapes take turns)."""
    per = {sh: [] for sh in shapes}
    handle.set_profiling(1)
    for _ in range(rounds):
        for sh in shapes:
            handle.set_tiles(*sh)
            handle.step(1)  # a first step on the shape, untimed (new kernels warm)
            handle.step(steps)
            ms, n = handle.stage_times()
            per[sh].append(sum(ms[k] for k in ANNIHILATION_STAGES) / max(n, 1))
    handle.set_profiling(0)
    return {sh: float(np.median(v)) for sh, v in per.items()}


def tune(handle, kb, label, shapes=SHAPES, steps=20, rounds=3):
    """One table row from a handle at its list of interest: the fastest shape."""
    n_entries = handle.list_size()
    t = time_shapes(handle, shapes, steps, rounds)
    best = min(t, key=t.get)
    return dict(label=label, key_bytes=kb, n_entries=int(n_entries), sort_it=best[0],
                merge_it=best[1], ms={f"{s}x{m}": round(v, 5) for (s, m), v in t.items()})


def write_table(rows, path=TABLE):
    """Table rows by key width, ascending in list size; a row applies from the
    geometric middle between its tuned size and the previous one."""
    out = {"version": 1, "rows": {}, "runs": rows}
    for kb in sorted({r["key_bytes"] for r in rows}):
        rs = sorted((r for r in rows if r["key_bytes"] == kb), key=lambda r: r["n_entries"])
        table = []
        for i, r in enumerate(rs):
            lo = 0 if i == 0 else int(math.sqrt(rs[i - 1]["n_entries"] * r["n_entries"]))
            if table and lo <= table[-1][0]:
                continue
            table.append([lo, r["sort_it"], r["merge_it"]])
        out["rows"][f"k{kb}"] = table
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def load_table(path=TABLE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def apply(handle, kb, path=TABLE):
    """Give the handle the tuned rows for its key width; returns them ([] if the
    table has none, and the handle keeps its default shape)."""
    t = load_table(path)
    rows = [] if t is None else t["rows"].get(f"k{kb}", [])
    if rows:
        handle.set_tile_table([tuple(r) for r in rows])
    return rows
