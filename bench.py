"""Benchmark of the DDQMC propagation step on one MI355X.

Workload: the 4x4 periodic dissipative XYZ lattice (Jx 0.9, Jy 1, Jz 1, gamma 1,
dt 0.002, initiator n_a 3, importance sampling p = 1.5) started with 1e7 real
walkers on |dn..dn><dn..dn|, the population the shift then holds.  W warm-up
steps, then K timed steps.  A "step" is one pass of the whole path: spawn and
clone/death, the radix sort of the spawn records, the merge/annihilation with
the initiator rule and the estimator sums, and the shift update.

Metric: walker-updates/s = sum over the timed steps of W_tot at the start of the
step (|re| + |im| summed over the list) / wall time.  Also reported: the
roofline position of the kernel that takes most of the step time (algorithmic
bytes per launch / its mean duration from HIP events on the handle's stream),
and the CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--steps K] [--warmup W] [--workload d3|d3l] [--no-cpu]
       python bench.py --workload d5 [--steps K]    (64 5x5 replicas, batched vs one by one)
       python bench.py --workload d4 [--requests R]  (serving loop vs one solve at a time)
       python bench.py --trace-summary DIR --steps K
The second form reads the kernel trace rocprofv3 wrote into DIR for a run of the
first form and prints, per kernel, the mean dispatch duration over the last K
steps (the timed region) as a markdown table.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
VALU_PEAK_G = 256 * 4 * 2.4 / 4  # G wave64 VALU instructions/s: 256 CUs x 4 SIMDs, 4 cycles each
PROF_EVERY = 10  # timed steps per step with stage events
KEY_BYTES = {True: 8, False: 4}

WORKLOADS = {
    "d3": (dict(workloads.D3),
           "4x4 periodic dissipative XYZ, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, n_a 3, "
           "IS p 1.5, 1e7 walkers"),
    # same physics, population raised so the walker list outgrows the 256 MB
    # last-level cache
    "d3l": (dict(workloads.D3, target_walkers=400_000_000, initial_walkers=400_000_000),
            "4x4 periodic dissipative XYZ, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, n_a 3, "
            "IS p 1.5, 4e8 walkers"),
}


def kernel_source_hash(texts=None):
    """Hash of the kernel sources with comments and blank space removed, so that
    a counter record stays valid across comment-only edits."""
    h = hashlib.sha256()
    for f in ("kernels.hpp", "model.hpp", "sampling.hpp", "ddqmc.hip"):
        if texts is None:
            with open(os.path.join(ROOT, "paper_1802_05931_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = texts[f]
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        h.update("".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload, per_launch_alg):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def valu_from_profile(kernel, workload):
    """VALU wave-instructions per launch from the committed counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("valu_per_launch")


def cpu_baseline(cfg, keys, re, im, sc, budget_s=15.0):
    """The oracle as it stands, single-threaded, stepping the workload from the
    GPU's state for about budget_s seconds."""
    from oracle import orc
    orc.build(force=False)
    o = orc.Oracle(**cfg)
    o.set_list(keys, re, im)
    o.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
    w_start = int(abs(re.astype("int64")).sum() + abs(im.astype("int64")).sum())
    walker_updates = 0
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        walker_updates += w_start
        w_start = o.last()["w_tot"]
        steps += 1
    dt = time.perf_counter() - t0
    return dict(value=walker_updates / dt, unit="walker-updates/s", cores=1, kind="oracle",
                sample=f"{steps} oracle steps of the same workload from the GPU state at step "
                       f"{sc['step']} ({len(keys)} entries), {dt:.1f} s on one host core")


def trace_summary(directory, steps):
    """Per-kernel dispatch statistics of the last `steps` steps of a rocprofv3
    kernel trace (one k_finalize dispatch ends every step)."""
    import csv
    import glob
    files = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {directory}")
    rows = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                short = name.split("(")[0].replace("void ", "").replace("ddqmc::", "")
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short))
    rows.sort()
    fin = [i for i, r in enumerate(rows) if r[2].startswith("k_finalize")]
    if len(fin) < steps + 1:
        raise SystemExit(f"trace holds {len(fin)} steps, fewer than {steps} + 1")
    lo, hi = fin[-steps - 1] + 1, fin[-1] + 1
    stats = {}
    for t0, t1, name in rows[lo:hi]:
        d = stats.setdefault(name, [0, 0.0, float("inf"), 0.0])
        dur = (t1 - t0) / 1e3
        d[0] += 1
        d[1] += dur
        d[2] = min(d[2], dur)
        d[3] = max(d[3], dur)
    span = (rows[hi - 1][1] - rows[lo][0]) / 1e6
    out = [f"timed region: the last {steps} steps, {hi - lo} dispatches, "
           f"{span:.1f} ms from the first dispatch start to the last dispatch end", "",
           "| kernel | calls | calls/step | mean us | min us | max us | us/step |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for name, (n, tot, mn, mx) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| {name} | {n} | {n / steps:g} | {tot / n:.2f} | {mn:.2f} | {mx:.2f} | "
                   f"{tot / steps:.2f} |")
    print("\n".join(out))


def counter_summary(fetch_dir, write_dir, probe_mb, workload, valu_dir=None):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the step kernels from two
    rocprofv3 --pmc runs, scaled by what the same counters read for the probe
    kernel of known traffic (an elementwise add over probe_mb MiB: reads and
    writes probe_mb MiB).  Prints a markdown table and, for the merge kernels,
    the traffic records bench.py reads."""
    import csv
    import glob
    import collections

    def load(d, counter):
        fn = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not fn:
            raise SystemExit(f"no counter_collection.csv under {d}")
        vals = collections.defaultdict(list)
        for r in csv.DictReader(open(fn[0])):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("ddqmc::", "")
            vals[name].append(float(r["Counter_Value"]))
        return vals
    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    # the probe is the elementwise kernel that reads (the fill before it only writes)
    probe = [k for k in fetch if "elementwise" in k]
    if not probe:
        raise SystemExit("probe kernel not found in the counters")
    probe = [max(probe, key=lambda k: max(fetch[k]))]
    kib = probe_mb * 1024.0
    f_scale = kib / max(fetch[probe[0]])
    w_scale = kib / max(write[probe[0]])
    out = [f"FETCH_SIZE / WRITE_SIZE per dispatch; the probe (elementwise add over {probe_mb} MiB) "
           f"read {max(fetch[probe[0]]):.0f} KiB and wrote {max(write[probe[0]]):.0f} KiB, so the "
           f"scale factors are {f_scale:.4f} (fetch) and {w_scale:.4f} (write)", "",
           "| kernel | dispatches | fetch MB | write MB | HBM MB (scaled) |",
           "|---|---:|---:|---:|---:|"]
    rec = {}
    for name in sorted(fetch):
        if "elementwise" in name or name.startswith("__amd"):
            continue
        fm = sum(fetch[name]) / len(fetch[name]) * 1024 / 1e6
        wm = (sum(write[name]) / len(write[name]) * 1024 / 1e6) if name in write else 0.0
        tot = fm * f_scale + wm * w_scale
        out.append(f"| {name} | {len(fetch[name])} | {fm:.2f} | {wm:.2f} | {tot:.2f} |")
        rec[name] = tot * 1e6
    print("\n".join(out))
    for short, name in (("k_merge_write", "k_merge<unsigned int, true>"),
                        ("k_merge_count", "k_merge<unsigned int, false>"),
                        ("k_sort_pass", "k_sort_pass<unsigned int>"),
                        ("k_spawn_scan", "k_spawn_scan<unsigned int>"),
                        ("k_spawn_loud", "k_spawn_loud<unsigned int>")):
        if name in rec:
            path = os.path.join(ROOT, "profiles", f"{short}_{workload}_traffic.json")
            with open(path, "w") as f:
                json.dump({"bytes_per_launch": rec[name], "source_hash": kernel_source_hash(),
                           "fetch_scale": f_scale, "write_scale": w_scale}, f, indent=1)
            print(f"wrote {path}")
    if valu_dir:
        valu, waves = load(valu_dir, "SQ_INSTS_VALU"), load(valu_dir, "SQ_WAVES")
        print("\n| kernel | dispatches | waves | VALU wave-instructions |\n|---|---:|---:|---:|")
        best = {}  # per kernel, the instantiation with the most instructions per launch
        for name in sorted(valu):
            if "elementwise" in name or name.startswith("__amd"):
                continue
            v = sum(valu[name]) / len(valu[name])
            w = sum(waves[name]) / len(waves[name]) if name in waves else 0
            print(f"| {name} | {len(valu[name])} | {w:.0f} | {v:.0f} |")
            for short in ("k_spawn_loud", "k_spawn_heavy", "k_spawn_scan"):
                if name.startswith(short + "<unsigned int") and v > best.get(short, -1.0):
                    best[short] = v
        for short, v in best.items():
            path = os.path.join(ROOT, "profiles", f"{short}_{workload}_valu.json")
            with open(path, "w") as f:
                json.dump({"valu_per_launch": v, "source_hash": kernel_source_hash()}, f, indent=1)
            print(f"wrote {path}")


def _walker_updates(series, steps):
    """Sum of W_tot at the start of the last `steps` steps of a series."""
    import numpy as np
    import paper_1802_05931_amd as dq
    w = series[:, 3 + dq.SUM_NAMES.index("w_tot")].astype(np.float64)
    return float(w[-steps - 1:-1].sum())


def bench_d5(args):
    """64 independent 5x5 replicas: one batch handle (one launch per stage for
    all replicas) against the same replicas run one after another on their own
    handles.  The lists must come out identical."""
    import numpy as np
    import torch
    from paper_1802_05931_amd import serving
    steps = args.steps if args.steps != 1000 else 300
    cfgs = workloads.d5_replicas()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    print(f"d5: batched, {len(cfgs)} replicas x {steps} steps", file=sys.stderr, flush=True)
    gk = args.graph_steps
    tb, ob, lb = serving.replicas_batched(cfgs, steps, graph_k=gk, stream=stream)
    print(f"d5: batched {tb:.2f} s; sequential", file=sys.stderr, flush=True)
    ts, os_, ls = serving.replicas_sequential(
        cfgs, steps, graph_k=gk, stream=stream, log=lambda m: print(f"d5: {m}", file=sys.stderr, flush=True))
    print(f"d5: sequential {ts:.2f} s", file=sys.stderr, flush=True)
    same = all(len(a[0]) == len(c[0]) and all(np.array_equal(x, y) for x, y in zip(a, c))
               for a, c in zip(lb, ls))
    same_obs = all(a["acc"] == c["acc"] and a["step"] == c["step"] for a, c in zip(ob, os_))
    entries = int(sum(len(x[0]) for x in lb))
    out = {
        "metric": "replica-steps/s (64 x 5x5 XYZ replicas, batched)",
        "value": len(cfgs) * (steps - 1) / tb,
        "unit": "replica-steps/s",
        "n_gpus": 1, "steps": steps - 1, "warmup": 1,
        "ms_per_step": 1e3 * tb / (steps - 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32 walkers, f64 probabilities", "data": "synthetic",
        "config": {"workload": "64 replicas of the 5x5 dissipative XYZ model, Jx 0.5..1.2, "
                               "dt 0.002, n_a 3, p 0, targets log-uniform in [1e3, 2e4], "
                               "u64 keys",
                   "graph_steps": gk, "final_entries": entries},
        "sequential": {"seconds": ts, "value": len(cfgs) * (steps - 1) / ts},
        "batched_seconds": tb,
        "speedup_vs_sequential": ts / tb,
        "lists_identical": bool(same), "accumulators_identical": bool(same_obs),
        "mz": [round(o["mz"], 5) for o in ob[:8]],
    }
    print(json.dumps(out), flush=True)


def bench_d4(args):
    """The serving stream: Poisson arrivals at 20/s, mixed lattices and targets,
    continuous batching in one pool, against the same requests one at a time
    (every n-th request timed alone for exactly the steps it took in the pool:
    identical lists, so identical errors)."""
    import numpy as np
    import torch
    from paper_1802_05931_amd import serving
    reqs = workloads.d4_requests(count=args.requests)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    done = [0]

    def log(msg):
        done[0] += 1
        print(f"d4: {msg}", file=sys.stderr, flush=True)
    gk = args.graph_steps
    recs, ticks = serving.serve(reqs, graph_k=gk, stream=stream, log=log)
    wall = time.perf_counter() - t0
    lat = np.array([r["finished"] - r["arrival"] for r in recs])
    steps = np.array([r["steps"] for r in recs])
    conv = np.array([r["converged"] for r in recs])
    over = np.array([r["over_limit"] for r in recs])
    print(f"d4: served {len(recs)} in {wall:.1f} s; timing every {args.baseline_every}-th alone",
          file=sys.stderr, flush=True)
    alone = []
    for i in range(0, len(reqs), args.baseline_every):
        dt, obs = serving.solve_alone(reqs[i]["params"], int(steps[i]), graph_k=gk,
                                      stream=stream)
        print(f"d4: request {i} alone: {dt:.2f} s for {steps[i]} steps", file=sys.stderr,
              flush=True)
        assert obs["step"] == steps[i]
        assert abs(obs["mz"] - recs[i]["mz"]) == 0.0 or (np.isnan(obs["mz"]) and
                                                        np.isnan(recs[i]["mz"]))
        alone.append(dt)
    alone_total = float(np.sum(alone)) * args.baseline_every
    last_arrival = max(r["arrival"] for r in reqs)
    out = {
        "metric": "served solves/s (D4 stream: 2x2/3x3/4x4/2x6, Poisson 20/s)",
        "value": len(recs) / wall,
        "unit": "solves/s",
        "n_gpus": 1, "steps": int(steps.sum()), "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32 walkers, f64 probabilities", "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, lattices uniform over 2x2/3x3/4x4/2x6, "
                               "Jx U[0.5,1.2], Jz U[0.8,1.2], gamma U[0.5,2], dt 0.005, n_a 3, "
                               "targets log-uniform [1e3,1e5], Poisson arrivals 20/s",
                   "slots": 64, "tick_steps": 50, "graph_steps": gk,
                   "admission": "pool list below 6e7 entries",
                   "stop": "SE(M_z) < 1e-3 after >= 512 accumulated steps, 2000 steps, or "
                           "more than 4e6 entries"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "wall_s": wall, "last_arrival_s": last_arrival, "ticks": ticks,
        "converged": int(conv.sum()), "over_memory_limit": int(over.sum()),
        "steps_per_solve_median": float(np.median(steps)),
        "one_at_a_time": {"seconds_estimated": alone_total,
                          "sample": f"every {args.baseline_every}-th request alone "
                                    f"({len(alone)} solves, scaled by {args.baseline_every})",
                          "solves_per_s": len(recs) / alone_total},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=15000)
    ap.add_argument("--workload", default="d3", choices=sorted(WORKLOADS) + ["d4", "d5"])
    ap.add_argument("--requests", type=int, default=512, help="d4: requests in the stream")
    ap.add_argument("--baseline-every", type=int, default=8,
                    help="d4: time every n-th request alone for the one-at-a-time baseline")
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="d4/d5: launch the steps as HIP graphs of this many steps (even; 0 = "
                         "one launch per kernel)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--trace-summary", metavar="DIR")
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="FETCH_DIR WRITE_DIR [VALU_DIR]: summarise rocprofv3 --pmc runs")
    ap.add_argument("--save-state", metavar="FILE",
                    help="write the solve's checkpoint after the warm-up")
    ap.add_argument("--load-state", metavar="FILE",
                    help="start from a checkpoint of the same workload instead of warming up")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB three times "
                         "(a plain copy kernel of known size for scaling memory counters)")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary, args.steps)
        return
    if args.counter_summary:
        d = args.counter_summary
        counter_summary(d[0], d[1], args.copy_probe_mb, args.workload,
                        d[2] if len(d) > 2 else None)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU sharding of the step is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_05931_amd as dq

    if args.workload == "d5":
        return bench_d5(args)
    if args.workload == "d4":
        return bench_d4(args)
    cfg, desc = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    blob = None
    if args.load_state:
        with open(args.load_state, "rb") as f:
            blob = f.read()
        # room for the loaded list to grow without a reallocation (16 bytes an entry)
        cfg = dict(cfg, capacity_hint=2 * (len(blob) // 16))
    g = dq.Solve(dq.make_params(**cfg), stream=stream)
    if blob is not None:
        g.set_state(blob)
        del blob
        args.warmup = g.scalars()["step"]
        _, re0, im0 = g.walkers()
        w0 = int(np.abs(re0.astype(np.int64)).sum() + np.abs(im0.astype(np.int64)).sum())
        del re0, im0
    else:
        # in chunks, with a line per chunk on stderr (large workloads warm up for minutes)
        done = 0
        while done < args.warmup:
            n = min(2000, args.warmup - done)
            g.step(n)
            done += n
            print(f"warm-up: {done} steps, {g.list_size()} entries", file=sys.stderr, flush=True)
    if args.save_state:
        with open(args.save_state, "wb") as f:
            f.write(g.get_state())
    # stage events on every PROF_EVERY-th timed step (an event costs a few
    # microseconds of its step; the sampled steps give the mean launch times)
    g.set_profiling(PROF_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    series = g.series()
    counts = g.step_counts()
    stage_ms, stage_steps = g.stage_times()
    assert stage_steps == (args.steps + PROF_EVERY - 1) // PROF_EVERY
    # the sampled steps' stage times, scaled to all timed steps
    stage_ms = {k: v * args.steps / stage_steps for k, v in stage_ms.items()}
    sums = {n: i + 3 for i, n in enumerate(dq.SUM_NAMES)}
    w_tot = series[:, sums["w_tot"]]
    # W_tot at the start of each timed step = W_tot after the previous step
    if len(w_tot) >= args.steps + 1:
        w_start = w_tot[-args.steps - 1:-1]
    else:  # started from a checkpoint: the first step starts from the loaded list
        w_start = np.concatenate([[w0], w_tot[:-1]])
    walker_updates = float(w_start.sum())
    c = counts[-args.steps:]
    n_in, n_sp, n_out = (c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float))
    k64 = 2 * cfg["Lx"] * cfg["Ly"] > 32
    rec = KEY_BYTES[k64] + 8  # key + (re, im) int32
    passes = (2 * cfg["Lx"] * cfg["Ly"] + 7) // 8
    alg_bytes = {  # what each kernel must read and write, per the step's counts
        # the list in, the loud entries out (index, key, value)
        "scan": float((n_in * rec + c[:, 3] * (rec + 4)).sum()),
        # per pass: the digit counts read the keys, the scatter reads and writes records
        "sort": float((passes * n_sp * (KEY_BYTES[k64] + 2 * rec)).sum()),
        # survivors per tile: the list's keys and the records
        "count": float((n_in * KEY_BYTES[k64] + n_sp * rec).sum()),
        # the list and the records in, the new list out
        "merge": float(((n_in + n_sp + n_out) * rec).sum()),
    }
    launches = {"scan": args.steps, "sort": args.steps * passes,
                "count": args.steps, "merge": args.steps}
    kernel_names = {"scan": "k_spawn_scan", "sort": "k_sort_pass",
                    "count": "k_merge_count", "merge": "k_merge_write"}
    # HBM roofline of the merge (the annihilation join, where the list is
    # streamed in and out): algorithmic bytes / mean launch time
    m_dur = stage_ms["merge"] / 1e3 / launches["merge"]
    m_bytes = alg_bytes["merge"] / launches["merge"]
    m_ach = m_bytes / m_dur / 1e9
    hbm_roofline = dict(kernel="k_merge_write", bound="hbm", achieved=round(m_ach, 1),
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=round(m_ach / HBM_PEAK_GBS, 4),
                        traffic=traffic_from_profile("k_merge_write", args.workload, m_bytes),
                        bytes_per_launch=round(m_bytes), mean_launch_us=round(m_dur * 1e6, 2))
    # the annihilation stages together (sort, merge count, merge write) on
    # their algorithmic bytes, and the method's minimal traffic per step
    # (read and write the list, write the records and read them back)
    a_stages = ("sort", "count", "merge")
    a_bytes = sum(alg_bytes[k] for k in a_stages)
    a_s = sum(stage_ms[k] for k in a_stages) / 1e3
    a_ach = a_bytes / a_s / 1e9
    b_alg = float((2 * n_in * rec + 2 * n_sp * (rec + 1)).sum()) / args.steps
    annihilation = dict(stages=list(a_stages), bytes_per_step=round(a_bytes / args.steps),
                        achieved=round(a_ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(a_ach / HBM_PEAK_GBS, 4),
                        method_min_bytes_per_step=round(b_alg))
    # the dominant kernel by time
    dominant = max((k for k in stage_ms if k != "finalize"), key=lambda k: stage_ms[k])
    if dominant in alg_bytes:
        dur_s = stage_ms[dominant] / 1e3 / launches[dominant]
        per_launch = alg_bytes[dominant] / launches[dominant]
        achieved = per_launch / dur_s / 1e9
        roofline = dict(kernel=kernel_names[dominant], bound="hbm", achieved=round(achieved, 1),
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=traffic_from_profile(kernel_names[dominant], args.workload,
                                                     per_launch),
                        bytes_per_launch=round(per_launch), mean_launch_us=round(dur_s * 1e6, 2))
    else:
        # a sampling kernel: bound by vector ALU issue, measured as VALU
        # instructions per launch (committed counter profile) over the live launch
        # time, against 256 CUs x 4 SIMDs issuing one wave64 instruction per 4
        # cycles at 2.4 GHz
        kname = {"loud": "k_spawn_loud", "heavy": "k_spawn_heavy"}.get(dominant, dominant)
        dur_s = stage_ms[dominant] / 1e3 / args.steps
        valu = valu_from_profile(kname, args.workload)
        achieved = valu / dur_s / 1e9 if valu else None
        roofline = dict(kernel=kname, bound="alu", achieved=(round(achieved, 1) if achieved
                                                              else None),
                        peak=VALU_PEAK_G, unit="G VALU wave-instructions/s",
                        frac=(round(achieved / VALU_PEAK_G, 4) if achieved else None),
                        traffic=traffic_from_profile(kname, args.workload, 0),
                        valu_instructions_per_launch=valu, mean_launch_us=round(dur_s * 1e6, 2))
    stages = {k: dict(ms_per_step=round(v / args.steps, 5),
                      achieved_GBs=(round(alg_bytes[k] / (v / 1e3) / 1e9, 1)
                                    if k in alg_bytes and v > 0 else None))
              for k, v in stage_ms.items()}
    keys, re, im = g.walkers()
    sc = g.scalars()
    obs = g.observables()
    out = {
        "metric": "walker-updates/s (4x4 XYZ)",
        "value": walker_updates / wall,
        "unit": "walker-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32 walkers, f64 probabilities",
        "data": "synthetic",
        "config": {"workload": desc, "lattice": "4x4", "target_walkers": cfg["target_walkers"],
                   "key_bits": 2 * cfg["Lx"] * cfg["Ly"], "mean_entries": float(n_in.mean()),
                   "mean_walkers": float(w_start.mean()),
                   "mean_spawn_records": float(n_sp.mean()),
                   "mean_loud_entries": float(c[:, 3].mean()),
                   "mean_heavy_entries": float(c[:, 4].mean())},
        "entry_updates_per_s": float(n_in.sum()) / wall,
        "roofline": roofline,
        "hbm_roofline": hbm_roofline,
        "hbm_annihilation": annihilation,
        "stages": stages,
        "stage_events": f"HIP events on every {PROF_EVERY}-th timed step ({stage_steps} steps)",
        "shift": sc["S"],
        "mz_running": obs["mz"],
    }
    g.set_profiling(False)
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):  # reads and writes copy_probe_mb MiB each
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, keys, re, im, sc, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
