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
       python bench.py --trace-summary DIR --steps K
The second form reads the kernel trace rocprofv3 wrote into DIR for a run of the
first form and prints, per kernel, the mean dispatch duration over the last K
steps (the timed region) as a markdown table.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "model.hpp", "sampling.hpp", "ddqmc.hip"):
        with open(os.path.join(ROOT, "paper_1802_05931_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=15000)
    ap.add_argument("--workload", default="d3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--trace-summary", metavar="DIR")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary, args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the "
              "multi-GPU sharding of the step is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_05931_amd as dq

    cfg, desc = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    g = dq.Solve(dq.make_params(**cfg), stream=stream)
    g.step(args.warmup)
    g.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    series = g.series()
    counts = g.step_counts()
    stage_ms, stage_steps = g.stage_times()
    assert stage_steps == args.steps
    sums = {n: i + 3 for i, n in enumerate(dq.SUM_NAMES)}
    w_tot = series[:, sums["w_tot"]]
    # W_tot at the start of each timed step = W_tot after the previous step
    w_start = w_tot[-args.steps - 1:-1]
    walker_updates = float(w_start.sum())
    c = counts[-args.steps:]
    n_in, n_sp, n_out = (c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float))
    k64 = 2 * cfg["Lx"] * cfg["Ly"] > 32
    rec = KEY_BYTES[k64] + 8  # key + (re, im) int32
    passes = (2 * cfg["Lx"] * cfg["Ly"] + 7) // 8
    alg_bytes = {  # what each kernel must read and write, per the step's counts
        "scan": float((n_in * rec).sum()),
        "histogram": float((n_sp * KEY_BYTES[k64]).sum()),
        "sort": float((2 * passes * n_sp * rec).sum()),
        # survivors per tile: the list's keys and the records
        "count": float((n_in * KEY_BYTES[k64] + n_sp * rec).sum()),
        # the list and the records in, the new list out
        "merge": float(((n_in + n_sp + n_out) * rec).sum()),
    }
    launches = {"scan": args.steps, "histogram": args.steps, "sort": args.steps * passes,
                "count": args.steps, "merge": args.steps}
    kernel_names = {"scan": "k_spawn_scan", "histogram": "k_hist", "sort": "k_sort_pass",
                    "count": "k_merge<count>", "merge": "k_merge<write>"}
    dominant = max(alg_bytes, key=lambda k: stage_ms[k])
    dur_s = stage_ms[dominant] / 1e3 / launches[dominant]
    per_launch = alg_bytes[dominant] / launches[dominant]
    achieved = per_launch / dur_s / 1e9
    traffic = traffic_from_profile(kernel_names[dominant], args.workload, per_launch)
    roofline = dict(kernel=kernel_names[dominant], bound="hbm", achieved=round(achieved, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic, bytes_per_launch=round(per_launch),
                    mean_launch_us=round(dur_s * 1e6, 2))
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
                   "mean_spawn_records": float(n_sp.mean())},
        "entry_updates_per_s": float(n_in.sum()) / wall,
        "roofline": roofline,
        "stages": stages,
        "shift": sc["S"],
        "mz_running": obs["mz"],
    }
    g.set_profiling(False)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, keys, re, im, sc, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
