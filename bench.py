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

Before the W warm-up steps the solve is always brought to its steady list:
it is stepped in chunks of 500 until the list size changes by less than 1%
over the last 1000 steps (at least 2000 steps; the 4x4 list settles at about
1.1e7 entries after some 14,000 steps), so that the timed steps see the
workload's own list and not the start-up transient.

The default line also carries the two systems forms beside the plain step:
"batched" (64 5x5 replicas in one batch handle against the same replicas one
after another) and "served" (the 512-request serving stream against the same
requests one at a time), each with its own timing and equal-error check.

Usage: python bench.py [--steps K] [--warmup W] [--workload d3|d3l|d3f|d3big] [--no-cpu]
                       [--legs d3,d5,d4]
       python bench.py --workload d5 [--steps K]    (64 5x5 replicas, batched vs one by one)
       python bench.py --workload d4 [--requests R]  (serving loop vs one solve at a time)
       python bench.py --workload perwalker [--steps K]  (per-walker vs per-entry sampling)
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
# (record name, start of the kernel name in the rocprofv3 output) of the
# 32-bit-key step kernels whose counter records bench.py reads; the tile shape
# follows in the template arguments (", 8>"), and of several instantiations the
# one that moved the most bytes is the workload's
KERNEL_RECORDS = (("k_merge_write", "k_merge<unsigned int, true"),
                  ("k_merge_count", "k_merge<unsigned int, false"),
                  ("k_sort_pass", "k_sort_pass<unsigned int"),
                  ("k_sort_count", "k_sort_count<unsigned int"),
                  ("k_merge_partition", "k_merge_partition<unsigned int"),
                  ("k_spawn_scan", "k_spawn_scan<unsigned int"),
                  ("k_spawn_loud", "k_spawn_loud<unsigned int"))
EQUIL_CHUNK = 500    # steps per equilibration chunk
EQUIL_MIN = 2000     # equilibration steps at least
EQUIL_MAX = 40000    # and at most
EQUIL_TOL = 0.01     # steady: the list changed by less than this over the last two chunks

WORKLOADS = {
    "d3": (dict(workloads.D3),
           "4x4 periodic dissipative XYZ, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, n_a 3, "
           "IS p 1.5, 1e7 walkers"),
    # no initiator: the list grows without a steady size (past 2e8 entries
    # within ~750 steps at 1e6 walkers); timed as it passes 1e8 entries
    # (1.2 GB of list), far beyond the 256 MB last-level cache
    "d3big": (dict(workloads.D3, n_a=0),
              "4x4 periodic dissipative XYZ, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, no initiator, "
              "IS p 1.5, 1e7 walkers, timed as its growing list passes 1e8 entries"),
    # the in-plane field along x (Sec. V.B): the parity rule no longer holds,
    # the list grows to about 7.7e7 entries, and the spawns go through the
    # field's sampling routines
    "d3f": (dict(workloads.D3, hx=0.05),
            "4x4 periodic dissipative XYZ, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, n_a 3, "
            "IS p 1.5, in-plane field hx 0.05, 1e7 walkers"),
    # same physics and population without importance sampling: the list holds
    # more configurations (the occupancy census at 1e6 walkers: 1.06e7 against
    # 6.1e6 with p 1.5; here about 1.38e7), 165 MB per list buffer, so its two
    # buffers outgrow the 256 MB last-level cache
    "d3l": (dict(workloads.D3, is_p=0.0),
            "4x4 periodic dissipative XYZ, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, n_a 3, "
            "no IS, 1e7 walkers"),
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


STATE_TOL = 0.10  # a counter record applies to live means within 10% of its own


def profile_record(kernel, workload, kind, live=None):
    """The committed rocprofv3 counter record ``profiles/<kernel>_<workload>_<kind>.json``
    (kind "traffic" or "valu") if it was taken on the current kernel sources and,
    when ``live`` is given, on a workload state like the live one: its mean list
    entries and mean spawn records per step within 10% of the live means.  A
    record taken on another state (another list size) says nothing about this
    run's launches, so it is not used.  Else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{kind}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    if live is not None:
        for k in ("mean_entries", "mean_spawn_records"):
            ref = d.get(k)
            if not ref or abs(float(live[k]) - float(ref)) > STATE_TOL * float(ref):
                return None
    return d


def traffic_from_profile(kernel, workload, live=None):
    """HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) from the committed
    counter record, or None (see profile_record)."""
    d = profile_record(kernel, workload, "traffic", live)
    return None if d is None else d.get("bytes_per_launch")


def valu_from_profile(kernel, workload, live=None):
    """VALU wave-instructions per launch from the committed counter record, or
    None (see profile_record)."""
    d = profile_record(kernel, workload, "valu", live)
    return None if d is None else d.get("valu_per_launch")


def _oracle_steps(cfg, keys, re, im, sc, budget_s):
    """Step the oracle from a list and its scalars for about budget_s seconds:
    (walker-updates, entry-updates, steps, seconds)."""
    from oracle import orc
    o = orc.Oracle(**cfg)
    o.set_list(keys, re, im)
    o.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
    w_start = int(abs(re.astype("int64")).sum() + abs(im.astype("int64")).sum())
    n_start = len(keys)
    walker_updates = entry_updates = steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        walker_updates += w_start
        entry_updates += n_start
        w_start = o.last()["w_tot"]
        n_start = o.size()
        steps += 1
    dt = time.perf_counter() - t0
    o.close()
    return walker_updates, entry_updates, steps, dt


def host_cpus():
    """The host's processor model, its logical CPU count and the CPUs this
    process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, nproc=os.cpu_count(), usable=sorted(os.sched_getaffinity(0)))


def cpu_baseline(cfg, keys, re, im, sc, budget_s=15.0, workers=None):
    """The oracle as it stands, single-threaded, stepping the workload from the
    GPU's state for about budget_s seconds; then the same sample on `workers`
    cores at once (default: every usable CPU, at most 16), one oracle process
    per core with a seed of its own, as the all-cores aggregate."""
    from oracle import orc
    orc.build(force=False)
    wu, eu, steps, dt = _oracle_steps(cfg, keys, re, im, sc, budget_s)
    host = host_cpus()
    out = dict(value=wu / dt, unit="walker-updates/s", cores=1, kind="oracle",
               entry_updates_per_s=eu / dt,
               sample=f"{steps} oracle steps of the same workload from the GPU state at step "
                      f"{sc['step']} ({len(keys)} entries), {dt:.1f} s on one host core",
               host=dict(model=host["model"], nproc=host["nproc"],
                         usable_cpus=len(host["usable"])))
    if workers is None:
        workers = min(16, len(host["usable"]))
    if workers > 1:
        out["all_cores"] = cpu_aggregate(cfg, keys, re, im, sc, budget_s, host["usable"][:workers])
    return out


def cpu_aggregate(cfg, keys, re, im, sc, budget_s, cpus):
    """The oracle sample in one process per CPU of `cpus`, all at once, each
    pinned to its CPU and with its own seed: the sum of their rates."""
    import subprocess
    import tempfile
    import numpy as np
    with tempfile.TemporaryDirectory() as d:
        np.savez(os.path.join(d, "list.npz"), keys=keys, re=re, im=im)
        with open(os.path.join(d, "job.json"), "w") as f:
            json.dump(dict(cfg=cfg, sc=sc, budget_s=budget_s), f)
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", d,
                                   "--cpu-seed", str(i + 1), "--cpu-core", str(c)],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
                 for i, c in enumerate(cpus)]
        res = []
        try:
            for p in procs:
                o, e = p.communicate()
                if p.returncode != 0:
                    raise RuntimeError(f"oracle worker failed ({p.returncode}): {e[-400:]}")
                res.append(json.loads(o.strip().splitlines()[-1]))
        finally:  # no worker outlives a failed one
            for p in procs:
                if p.poll() is None:
                    p.kill()
                    p.wait()
    steps = [r["steps"] for r in res]
    return dict(value=sum(r["walker_updates"] / r["seconds"] for r in res),
                unit="walker-updates/s", cores=len(cpus),
                entry_updates_per_s=sum(r["entry_updates"] / r["seconds"] for r in res),
                sample=f"{len(cpus)} oracle processes at once, each pinned to one host CPU, "
                       f"seeds 1..{len(cpus)}, each stepping the same GPU state for about "
                       f"{budget_s:g} s ({min(steps)}-{max(steps)} steps)")


def cpu_worker(directory, seed, core):
    """One process of the all-cores aggregate: prints its counts as JSON."""
    import numpy as np
    os.sched_setaffinity(0, {core})
    with open(os.path.join(directory, "job.json")) as f:
        job = json.load(f)
    z = np.load(os.path.join(directory, "list.npz"))
    cfg = dict(job["cfg"], seed=int(job["cfg"].get("seed", 0)) + seed)
    wu, eu, steps, dt = _oracle_steps(cfg, z["keys"], z["re"], z["im"], job["sc"],
                                      job["budget_s"])
    print(json.dumps(dict(walker_updates=wu, entry_updates=eu, steps=steps, seconds=dt)),
          flush=True)


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


def counter_summary(fetch_dir, write_dir, probe_mb, workload, valu_dir=None, state=None,
                    req_dir=None):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the step kernels from two
    rocprofv3 --pmc runs, scaled by what the same counters read for the probe
    kernel of known traffic (an elementwise add over probe_mb MiB: reads and
    writes probe_mb MiB).  Prints a markdown table and, for the step kernels,
    the traffic records bench.py reads.  ``state`` holds the mean list entries
    and spawn records per step of the profiled run (from its bench line); the
    records carry them, so that bench.py uses a record only on a like state.
    ``req_dir``, a third run with TCC_EA0_RDREQ_{32B,64B,128B}_sum, gives each
    kernel's read bytes from its own request sizes (32, 64 and 128 bytes), a
    cross-check of the one probe factor applied to every kernel."""
    state = {k: (state or {}).get(k) for k in ("mean_entries", "mean_spawn_records")}
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
    req = None
    if req_dir:
        c32, c64, c128 = (load(req_dir, f"TCC_EA0_RDREQ_{b}_sum") for b in ("32B", "64B", "128B"))

        def mean(d, k):
            return sum(d[k]) / len(d[k]) if d.get(k) else 0.0
        req = {k: 32 * mean(c32, k) + 64 * mean(c64, k) + 128 * mean(c128, k) for k in c32}
        pk = [k for k in req if "elementwise" in k]
        if pk:
            pr = max(req[k] for k in pk)
            out[0] += (f"; by request sizes the probe read {pr / 2 ** 20:.1f} MiB "
                       f"(of {probe_mb} MiB)")
        out[2] = out[2] + " read MB by request size | HBM MB (request sizes) |"
        out[3] = out[3] + "---:|---:|"
    rec, rec_req = {}, {}
    for name in sorted(fetch):
        if "elementwise" in name or name.startswith("__amd"):
            continue
        fm = sum(fetch[name]) / len(fetch[name]) * 1024 / 1e6
        wm = (sum(write[name]) / len(write[name]) * 1024 / 1e6) if name in write else 0.0
        tot = fm * f_scale + wm * w_scale
        line = f"| {name} | {len(fetch[name])} | {fm:.2f} | {wm:.2f} | {tot:.2f} |"
        rec[name] = tot * 1e6
        if req is not None:
            rm = req.get(name, 0.0) / 1e6
            rec_req[name] = (rm + wm) * 1e6
            line += f" {rm:.2f} | {rm + wm:.2f} |"
        out.append(line)
    print("\n".join(out))
    for short, prefix in KERNEL_RECORDS:
        names = [n for n in rec if n.startswith(prefix)]
        if not names:
            continue
        name = max(names, key=lambda n: rec[n])
        path = os.path.join(ROOT, "profiles", f"{short}_{workload}_traffic.json")
        d = {"kernel": name, "bytes_per_launch": rec[name], "source_hash": kernel_source_hash(),
             "fetch_scale": f_scale, "write_scale": w_scale}
        if name in rec_req:
            d["bytes_per_launch_by_request_size"] = rec_req[name]
        with open(path, "w") as f:
            json.dump(dict(d, **state), f, indent=1)
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
                json.dump(dict({"valu_per_launch": v, "source_hash": kernel_source_hash()},
                               **state), f, indent=1)
            print(f"wrote {path}")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def equilibrate(g, log=_log):
    """Steps a solve in chunks of EQUIL_CHUNK until its list is steady: at
    least EQUIL_MIN steps, and the list size changed by less than EQUIL_TOL
    over the last two chunks.  Returns (steps taken, steady, list sizes)."""
    sizes = []
    done = 0
    while done < EQUIL_MAX:
        g.step(EQUIL_CHUNK)
        done += EQUIL_CHUNK
        sizes.append(g.list_size())
        log(f"equilibration: {done} steps, {sizes[-1]} entries")
        if (done >= EQUIL_MIN and len(sizes) >= 3
                and abs(sizes[-1] - sizes[-3]) <= EQUIL_TOL * sizes[-1]):
            return done, True, sizes
    return done, False, sizes


def bench_d5(args, log=_log):
    """64 independent 5x5 replicas: one batch handle (one launch per stage for
    all replicas) against the same replicas run one after another on their own
    handles.  The lists must come out identical (so the statistical error is
    the same by construction)."""
    import numpy as np
    import torch
    from paper_1802_05931_amd import serving
    steps = args.d5_steps
    cfgs = workloads.d5_replicas()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    log(f"d5: batched, {len(cfgs)} replicas x {steps} steps")
    gk = args.graph_steps
    from paper_1802_05931_amd import autotune
    t = None if args.no_tuned else autotune.load_table()
    rows = [] if t is None else t["rows"].get("k8", [])  # 5x5: 50-bit keys, alone or batched
    tb, ob, lb = serving.replicas_batched(cfgs, steps, graph_k=gk, stream=stream, tile_rows=rows)
    log(f"d5: batched {tb:.2f} s; sequential")
    ts, os_, ls = serving.replicas_sequential(
        cfgs, steps, graph_k=gk, stream=stream, log=lambda m: log(f"d5: {m}"), tile_rows=rows)
    log(f"d5: sequential {ts:.2f} s")
    same = all(len(a[0]) == len(c[0]) and all(np.array_equal(x, y) for x, y in zip(a, c))
               for a, c in zip(lb, ls))
    same_obs = all(a["acc"] == c["acc"] and a["step"] == c["step"] for a, c in zip(ob, os_))
    entries = int(sum(len(x[0]) for x in lb))
    return {
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
                   "graph_steps": gk, "final_entries": entries, "tile_table": rows},
        "sequential": {"seconds": ts, "value": len(cfgs) * (steps - 1) / ts},
        "batched_seconds": tb,
        "speedup_vs_sequential": ts / tb,
        "equal_error": "lists and accumulators identical batched and alone",
        "lists_identical": bool(same), "accumulators_identical": bool(same_obs),
        "se_mz": [float(o["se_mz"]) for o in ob[:4]],
        "mz": [round(o["mz"], 5) for o in ob[:8]],
    }


def bench_d4(args, log=_log):
    """The serving stream: Poisson arrivals at 20/s, mixed lattices and targets,
    continuous batching in one pool, against the same requests one at a time
    (every n-th request timed alone for exactly the steps it took in the pool:
    identical lists, so identical errors)."""
    import numpy as np
    import torch
    from paper_1802_05931_amd import serving
    reqs = workloads.d4_requests(count=args.requests, t_hi=args.d4_target_max)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    gk = args.graph_steps
    recs, st = serving.serve(reqs, graph_k=gk, stream=stream, log=lambda m: log(f"d4: {m}"))
    ticks = st["ticks"]
    wall = time.perf_counter() - t0
    lat = np.array([r["finished"] - r["arrival"] for r in recs])
    steps = np.array([r["steps"] for r in recs])
    conv = np.array([r["converged"] for r in recs])
    over = np.array([r["over_limit"] for r in recs])
    log(f"d4: served {len(recs)} in {wall:.1f} s; timing every {args.baseline_every}-th alone")
    alone = []
    for i in range(0, len(reqs), args.baseline_every):
        dt, obs = serving.solve_alone(reqs[i]["params"], int(steps[i]), graph_k=gk,
                                      stream=stream)
        log(f"d4: request {i} alone: {dt:.2f} s for {steps[i]} steps")
        assert obs["step"] == steps[i]
        assert obs["mz"] == recs[i]["mz"] or (np.isnan(obs["mz"]) and np.isnan(recs[i]["mz"]))
        assert obs["se_mz"] == recs[i]["se_mz"] or (np.isnan(obs["se_mz"]) and
                                                    np.isnan(recs[i]["se_mz"]))
        alone.append(dt)
    alone_total = float(np.sum(alone)) * args.baseline_every
    last_arrival = max(r["arrival"] for r in reqs)
    return {
        "metric": "served solves/s (D4 stream: 2x2/3x3/4x4/2x6, Poisson 20/s)",
        "value": len(recs) / wall,
        "unit": "solves/s",
        "n_gpus": 1, "steps": int(steps.sum()), "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32 walkers, f64 probabilities", "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, lattices uniform over 2x2/3x3/4x4/2x6, "
                               "Jx U[0.5,1.2], Jz U[0.8,1.2], gamma U[0.5,2], dt 0.005, n_a 3, "
                               f"targets log-uniform [1e3,{args.d4_target_max:.0e}], "
                               "Poisson arrivals 20/s",
                   "slots": 64, "tick_steps": 50, "graph_steps": gk,
                   "admission": "in arrival order while the projected device bytes of the "
                                "admitted solves (the workspace of min(reachable "
                                "configurations, 4e6) entries each) stay within 32 GiB",
                   "max_active": st["max_active"],
                   "max_projected_GiB": round(st["max_projected_bytes"] / 2 ** 30, 2),
                   "evicted": st["evicted"],
                   "stop": "SE(M_z) < 1e-3 after >= 512 accumulated steps, 2000 steps, or "
                           "more than 4e6 entries"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "wall_s": wall, "last_arrival_s": last_arrival, "ticks": ticks,
        "converged": int(conv.sum()), "over_memory_limit": int(over.sum()),
        "steps_per_solve_median": float(np.median(steps)),
        "equal_error": "every timed alone solve has the pool's M_z and SE(M_z), bit for bit",
        "one_at_a_time": {"seconds_estimated": alone_total,
                          "sample": f"every {args.baseline_every}-th request alone "
                                    f"({len(alone)} solves, scaled by {args.baseline_every})",
                          "solves_per_s": len(recs) / alone_total},
    }


def bench_d3(args, log=_log):
    """The plain step on the 4x4 workload (or its large-list variant), timed on
    its steady list.  Returns (bench line without cpu_baseline, handle, cfg)."""
    import numpy as np
    import torch

    import paper_1802_05931_amd as dq

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
    from paper_1802_05931_amd import autotune
    tile_rows = [] if args.no_tuned else autotune.apply(g, autotune.key_bytes(cfg["Lx"] * cfg["Ly"]))
    if blob is not None:
        g.set_state(blob)
        del blob
        equil_steps, steady = g.scalars()["step"], True
        log(f"loaded state at step {equil_steps}, {g.list_size()} entries")
    elif args.workload == "d3big":
        # no steady list: step until it passes 1e8 entries
        equil_steps, steady = 0, False
        while g.list_size() < 100_000_000 and equil_steps < 5000:
            g.step(25)
            equil_steps += 25
            log(f"growth: {equil_steps} steps, {g.list_size()} entries")
    else:
        equil_steps, steady, _ = equilibrate(g, log)
    if args.save_state:
        with open(args.save_state, "wb") as f:
            f.write(g.get_state())
    if args.warmup:
        g.step(args.warmup)
    log(f"warm-up: {args.warmup} steps after {equil_steps} equilibration steps, "
        f"{g.list_size()} entries")
    w0 = int(g.observables()["last"]["w_tot"])
    # stage events on every prof_every-th timed step (an event costs a few
    # microseconds of its step; the sampled steps give the mean launch times)
    prof_every = max(1, min(PROF_EVERY, args.steps // 10))
    g.set_profiling(prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    series = g.series()
    counts = g.step_counts()
    stage_ms, stage_steps = g.stage_times()
    # (a step that regrows the buffers restarts the sampling for the rest of
    # its chunk, so the count of sampled steps is read, not assumed)
    assert stage_steps >= 1
    # the sampled steps' stage times, scaled to all timed steps
    stage_ms = {k: v * args.steps / stage_steps for k, v in stage_ms.items()}
    sums = {n: i + 3 for i, n in enumerate(dq.SUM_NAMES)}
    w_tot = series[:, sums["w_tot"]]
    # W_tot at the start of each timed step = W_tot after the previous step
    w_start = np.concatenate([[w0], w_tot[-args.steps:-1]]) if args.steps > 1 else np.array([w0])
    walker_updates = float(w_start.sum())
    c = counts[-args.steps:]
    n_in, n_sp, n_out = (c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float))
    live = dict(mean_entries=float(n_in.mean()), mean_spawn_records=float(n_sp.mean()))
    k64 = 2 * cfg["Lx"] * cfg["Ly"] > 32
    kb = KEY_BYTES[k64]
    rec = kb + 8  # key + (re, im) int32
    passes = (2 * cfg["Lx"] * cfg["Ly"] + 7) // 8
    alg_bytes = {  # what each kernel must read and write, per the step's counts
        # the list in, the loud entries out (index, key, value)
        "scan": float((n_in * rec + c[:, 3] * (rec + 4)).sum()),
        # per pass: the digit counts read the keys, the scatter reads and writes records
        "sort": float((passes * n_sp * (kb + 2 * rec)).sum()),
        # survivors per tile: the list's keys and the records
        "count": float((n_in * kb + n_sp * rec).sum()),
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
                        traffic=traffic_from_profile("k_merge_write", args.workload, live),
                        bytes_per_launch=round(m_bytes), mean_launch_us=round(m_dur * 1e6, 2))
    # The annihilation stages together (sort, merge count, merge write: the
    # HBM-bound part of the step) on the method's algorithmic bytes B_alg: read
    # and write the list, write the records and read them back,
    #   B_alg = 2 n_main (k_B + 8) + 2 n_sp (k_B + 9)  per step,
    # and, beside it, on the implementation's own bytes (radix passes and the
    # count pass re-read records and keys).
    a_stages = ("sort", "count", "merge")
    a_impl = sum(alg_bytes[k] for k in a_stages)
    a_s = sum(stage_ms[k] for k in a_stages) / 1e3
    b_alg = float((2 * n_in * rec + 2 * n_sp * (rec + 1)).sum())
    a_ach = b_alg / a_s / 1e9
    a_traffic = [traffic_from_profile(kernel_names[k], args.workload, live) for k in a_stages]
    annihilation = dict(stages=list(a_stages), bound="hbm",
                        bytes_per_step=round(b_alg / args.steps),
                        achieved=round(a_ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(a_ach / HBM_PEAK_GBS, 4),
                        us_per_step=round(a_s / args.steps * 1e6, 2),
                        implementation_bytes_per_step=round(a_impl / args.steps),
                        implementation_frac=round(a_impl / a_s / 1e9 / HBM_PEAK_GBS, 4))
    # the dominant kernel by time
    dominant = max((k for k in stage_ms if k != "finalize"), key=lambda k: stage_ms[k])
    if dominant in alg_bytes:
        dur_s = stage_ms[dominant] / 1e3 / launches[dominant]
        per_launch = alg_bytes[dominant] / launches[dominant]
        achieved = per_launch / dur_s / 1e9
        roofline = dict(kernel=kernel_names[dominant], bound="hbm", achieved=round(achieved, 1),
                        peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=traffic_from_profile(kernel_names[dominant], args.workload, live),
                        bytes_per_launch=round(per_launch), mean_launch_us=round(dur_s * 1e6, 2))
    else:
        # a sampling kernel: bound by vector ALU issue, measured as VALU
        # instructions per launch (committed counter record of a like state)
        # over the live launch time, against 256 CUs x 4 SIMDs issuing one
        # wave64 instruction per 4 cycles at 2.4 GHz
        kname = {"loud": "k_spawn_loud", "heavy": "k_spawn_heavy"}.get(dominant, dominant)
        dur_s = stage_ms[dominant] / 1e3 / args.steps
        valu = valu_from_profile(kname, args.workload, live)
        achieved = valu / dur_s / 1e9 if valu else None
        roofline = dict(kernel=kname, bound="alu", achieved=(round(achieved, 1) if achieved
                                                              else None),
                        peak=VALU_PEAK_G, unit="G VALU wave-instructions/s",
                        frac=(round(achieved / VALU_PEAK_G, 4) if achieved else None),
                        traffic=traffic_from_profile(kname, args.workload, live),
                        valu_instructions_per_launch=valu, mean_launch_us=round(dur_s * 1e6, 2))
    stages = {k: dict(ms_per_step=round(v / args.steps, 5),
                      achieved_GBs=(round(alg_bytes[k] / (v / 1e3) / 1e9, 1)
                                    if k in alg_bytes and v > 0 else None))
              for k, v in stage_ms.items()}
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
                   "key_bits": 2 * cfg["Lx"] * cfg["Ly"],
                   "equilibration_steps": int(equil_steps), "steady": bool(steady),
                   "mean_entries": live["mean_entries"],
                   "list_drift_over_timed_steps": float((n_in[-1] - n_in[0]) / n_in.mean()),
                   "mean_walkers": float(w_start.mean()),
                   "mean_spawn_records": live["mean_spawn_records"],
                   "mean_loud_entries": float(c[:, 3].mean()),
                   "mean_heavy_entries": float(c[:, 4].mean()),
                   "tile_table": tile_rows, "tiles_in_use": list(g.tiles())},
        "entry_updates_per_s": float(n_in.sum()) / wall,
        "bytes_per_walker_update": b_alg / walker_updates,
        "roofline": roofline,
        "hbm_roofline": hbm_roofline,
        "hbm_annihilation": annihilation,
        "stages": stages,
        "stage_events": f"HIP events on every {prof_every}-th timed step ({stage_steps} steps)",
        "shift": sc["S"],
        "mz_running": obs["mz"],
    }
    g.set_profiling(False)
    return out, g, cfg


def bench_perwalker(args, log=_log):
    """Ablation of the per-entry sampling: the 4x4 workload's steady list
    (equilibrated with the per-entry sampler, or loaded with --load-state)
    stepped from the same list and scalars by each sampler in turn -- per
    entry (all of an entry's walkers drawn at once, the default) and walker
    by walker (the rules of Sec. II, one thread per walker) -- W warm-up
    steps, then K timed steps each.  Both have the same expectation; the
    per-walker law spawns onto a uniformly chosen connection."""
    import numpy as np
    import torch

    import paper_1802_05931_amd as dq
    from paper_1802_05931_amd import autotune

    cfg, desc = WORKLOADS["d3"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    g = dq.Solve(dq.make_params(**cfg), stream=stream)
    if args.load_state:
        with open(args.load_state, "rb") as f:
            g.set_state(f.read())
        equil_steps = g.scalars()["step"]
    else:
        equil_steps, _, _ = equilibrate(g, log)
    keys, re, im = g.walkers()
    sc = g.scalars()
    g.close()
    log(f"perwalker: steady list of {len(keys)} entries after {equil_steps} steps")
    out = {}
    for name, flags in (("per_entry", 0), ("per_walker", dq.PER_WALKER)):
        h = dq.Solve(dq.make_params(**dict(cfg, flags=flags, capacity_hint=2 * len(keys))),
                     stream=stream)
        if not args.no_tuned:
            autotune.apply(h, autotune.key_bytes(cfg["Lx"] * cfg["Ly"]))
        h.set_walkers(keys, re, im)
        h.set_scalars(sc["S"], sc["mode"], sc["step"], sc["nw_prev"])
        h.step(args.warmup)
        w0 = int(h.observables()["last"]["w_tot"])
        h.set_profiling(max(1, min(PROF_EVERY, args.steps // 10)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.step(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        series = h.series()
        w_tot = series[:, 3 + list(dq.SUM_NAMES).index("w_tot")]
        w_start = np.concatenate([[w0], w_tot[-args.steps:-1]])
        c = h.step_counts()[-args.steps:]
        stage_ms, stage_steps = h.stage_times()
        spawn = sum(stage_ms[k] for k in ("scan", "gather", "loud", "heavy")) / stage_steps
        out[name] = dict(ms_per_step=1e3 * wall / args.steps,
                         walker_updates_per_s=float(w_start.sum()) / wall,
                         spawn_ms_per_step=round(spawn, 5),
                         mean_entries=float(c[:, 0].mean()),
                         mean_spawn_records=float(c[:, 1].mean()),
                         mean_walkers=float(w_start.mean()))
        log(f"perwalker: {name} {out[name]['ms_per_step']:.3f} ms/step, spawn "
            f"{out[name]['spawn_ms_per_step']:.3f} ms")
        h.set_profiling(False)
        h.close()
    pe, pw = out["per_entry"], out["per_walker"]
    return {
        "metric": "walker-updates/s (4x4 XYZ), per-walker sampling ablation",
        "value": pw["walker_updates_per_s"], "unit": "walker-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": pw["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i32 walkers, f64 probabilities", "data": "synthetic",
        "config": {"workload": desc + "; both samplers from the per-entry sampler's steady "
                                      "list", "equilibration_steps": int(equil_steps)},
        "per_entry": pe, "per_walker": pw,
        "per_entry_speedup": pw["ms_per_step"] / pe["ms_per_step"],
        "spawn_speedup": pw["spawn_ms_per_step"] / pe["spawn_ms_per_step"],
    }


def bench_tune(args, log=_log):
    """Tile-shape tuning (ddqmc_set_tiles): every shape timed on the 4x4
    workload's steady list, on smaller 4x4 and 3x3 lists, and on the 64-replica
    5x5 batch; the table goes to --tune-out (default the package's
    tuned_tiles.json)."""
    import torch

    import paper_1802_05931_amd as dq
    from paper_1802_05931_amd import autotune
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    runs = []

    def one(label, g, kb):
        r = autotune.tune(g, kb, label)
        log(f"tune {label}: {r['n_entries']} entries, best {r['sort_it']}x{r['merge_it']}: "
            f"{r['ms']}")
        runs.append(r)

    # 3x3 at its target of 1e5 walkers, and a 4x4 list of about 1e6 entries
    g = dq.Solve(dq.make_params(**workloads.d2(0.6)), stream=stream)
    g.step(3000)
    one("3x3 Jx 0.6, target 1e5", g, 4)
    g.close()
    g = dq.Solve(dq.make_params(**dict(workloads.D3, target_walkers=1_000_000,
                                       initial_walkers=1_000_000)), stream=stream)
    g.step(6000)
    one("4x4 target 1e6", g, 4)
    g.close()
    # the headline 4x4 list (steady, about 1.07e7 entries)
    g = dq.Solve(dq.make_params(**workloads.D3), stream=stream)
    equilibrate(g, log)
    one("4x4 target 1e7 (steady)", g, 4)
    g.close()
    # the 64-replica 5x5 batch after 250 of its 300 steps
    b = dq.Batch([dq.make_params(**c) for c in workloads.d5_replicas()], stream=stream)
    b.step(250)
    one("64 x 5x5 batch", b, 8)
    b.close()
    out = autotune.write_table(runs, args.tune_out or autotune.TABLE)
    print(json.dumps(out), flush=True)


def bench_census(args, log=_log):
    """Occupied configurations of the 4x4 workload's physics at 1e6 walkers, by
    initiator threshold and importance-sampling parameter (Sec. IV.B)."""
    import torch
    from paper_1802_05931_amd import studies
    torch.cuda.set_device(0)
    base = dict(workloads.D3, target_walkers=1_000_000, initial_walkers=1_000_000)
    grid = [(n, p) for p in (0.0, 1.5, 2.5) for n in (0, 3, 25, 75)]
    t0 = time.perf_counter()
    rows = studies.occupancy_census(base, grid, max_steps=args.census_steps, chunk=500,
                                    cap_limit=200_000_000, stream=torch.cuda.current_stream(),
                                    log=log)
    return {"study": "occupancy census (4x4, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, 1e6 walkers)",
            "rows": rows, "seconds": time.perf_counter() - t0}


def bench_extrapolate(args, log=_log):
    """The initiator extrapolation on the 4x4 workload's physics with the
    initiator figure's population and importance sampling (1e6 walkers, p 2.5):
    replicas at n_a = 3, 5, 8, 12 in one batch, M_z and C_yy read at n_a -> 0."""
    import torch
    from paper_1802_05931_amd import studies
    torch.cuda.set_device(0)
    base = dict(workloads.D3, target_walkers=1_000_000, initial_walkers=1_000_000, is_p=2.5,
                n_equil=args.extrap_steps // 2)
    t0 = time.perf_counter()
    recs = studies.initiator_runs(base, [3, 5, 8, 12], args.extrap_steps, graph_k=50,
                                  stream=torch.cuda.current_stream(), chunk=1000, log=log)
    for r in recs:
        log(f"extrapolate n_a {r['n_a']}: M_z {r['mz']:.5f} +- {r['se_mz']:.5f}, "
            f"C_yy {r['cyy']:.5f} +- {r['se_cyy']:.5f}, {r['entries']} entries")
    return {"study": "initiator extrapolation (4x4, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.002, "
                     "1e6 walkers, p 2.5)",
            "runs": recs, "mz": studies.extrapolate(recs, "mz"),
            "cyy": studies.extrapolate(recs, "cyy"), "steps": args.extrap_steps,
            "seconds": time.perf_counter() - t0}


def bench_susceptibility(args, log=_log):
    """One point of the angle-averaged susceptibility (Sec. V.B) on the 3x3
    lattice: the 3 + 3 + 1 field runs (h 0.01, 0.02, 0.03 along x and y, and
    none) in one batch, at the 3x3 workload's couplings and 1e5 walkers."""
    import torch
    from paper_1802_05931_amd import studies
    torch.cuda.set_device(0)
    base = dict(workloads.d2(0.9), target_walkers=100_000, initial_walkers=100_000,
                shift_init=0.0, n_equil=args.chi_steps // 4)
    t0 = time.perf_counter()
    r = studies.susceptibility(base, [0.01, 0.02, 0.03], args.chi_steps, graph_k=50,
                               stream=torch.cuda.current_stream(), chunk=2000, log=log)
    r.update(study="susceptibility (3x3, Jx 0.9 Jy 1 Jz 1 gamma 1, dt 0.005, n_a 3, 1e5 walkers)",
             steps=args.chi_steps, seconds=time.perf_counter() - t0)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20,
                    help="steps after the equilibration, before the timed steps")
    ap.add_argument("--workload", default="d3",
                    choices=sorted(WORKLOADS) + ["d4", "d5", "tune", "census", "extrapolate",
                                                 "susceptibility", "perwalker"])
    ap.add_argument("--chi-steps", type=int, default=20000,
                    help="susceptibility: steps of the 3 + 3 + 1 runs")
    ap.add_argument("--census-steps", type=int, default=20000,
                    help="census: most steps per run")
    ap.add_argument("--extrap-steps", type=int, default=16000,
                    help="extrapolate: steps of the batch (half of them accumulated)")
    ap.add_argument("--tune-out", metavar="FILE",
                    help="tune: where the tile table goes (default the package's table)")
    ap.add_argument("--no-tuned", action="store_true",
                    help="keep the default tile shapes instead of the tuned table")
    ap.add_argument("--legs", default="d3,d5,d4",
                    help="default line: the plain step (d3) and the batched (d5) and served "
                         "(d4) legs beside it")
    ap.add_argument("--requests", type=int, default=512, help="d4: requests in the stream")
    ap.add_argument("--d4-target-max", type=float, default=1e5,
                    help="d4: upper end of the log-uniform target walker range")
    ap.add_argument("--d5-steps", type=int, default=300, help="d5: steps per replica")
    ap.add_argument("--baseline-every", type=int, default=8,
                    help="d4: time every n-th request alone for the one-at-a-time baseline")
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="d4/d5: launch the steps as HIP graphs of this many steps (even; 0 = "
                         "one launch per kernel)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-cores", type=int, default=None,
                    help="processes of the oracle's all-cores aggregate (default: every "
                         "usable CPU, at most 16; 1 skips it)")
    ap.add_argument("--cpu-worker", metavar="DIR", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-seed", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-core", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--trace-summary", metavar="DIR")
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="FETCH_DIR WRITE_DIR [VALU_DIR [REQ_DIR]]: summarise rocprofv3 --pmc "
                         "runs")
    ap.add_argument("--bench-json", metavar="FILE",
                    help="with --counter-summary: the bench line of the profiled run (its "
                         "mean list entries and spawn records key the records)")
    ap.add_argument("--save-state", metavar="FILE",
                    help="write the solve's checkpoint after the equilibration")
    ap.add_argument("--load-state", metavar="FILE",
                    help="start from a checkpoint of the same workload instead of equilibrating")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB three times "
                         "(a plain copy kernel of known size for scaling memory counters)")
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.cpu_seed, args.cpu_core)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.steps)
        return
    if args.counter_summary:
        d = args.counter_summary
        state = None
        if args.bench_json:
            with open(args.bench_json) as f:
                line = [x for x in f.read().splitlines() if x.startswith("{")][-1]
            state = json.loads(line)["config"]
        counter_summary(d[0], d[1], args.copy_probe_mb, args.workload,
                        d[2] if len(d) > 2 else None, state, d[3] if len(d) > 3 else None)
        return
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU only (asked for {args.gpus}); its "
              "sharding over several GPUs is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.workload == "tune":
        bench_tune(args)
        return
    if args.workload == "census":
        print(json.dumps(bench_census(args)), flush=True)
        return
    if args.workload == "susceptibility":
        print(json.dumps(bench_susceptibility(args), default=float), flush=True)
        return
    if args.workload == "extrapolate":
        print(json.dumps(bench_extrapolate(args), default=float), flush=True)
        return
    if args.workload == "perwalker":
        print(json.dumps(bench_perwalker(args)), flush=True)
        return
    if args.workload == "d5":
        print(json.dumps(bench_d5(args)), flush=True)
        return
    if args.workload == "d4":
        print(json.dumps(bench_d4(args)), flush=True)
        return
    legs = [x for x in args.legs.split(",") if x]
    out, g, cfg = bench_d3(args)
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):  # reads and writes copy_probe_mb MiB each
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    keys, re, im = g.walkers()
    sc = g.scalars()
    g.close()
    del g
    if args.workload == "d3" and "d5" in legs:
        out["batched"] = bench_d5(args)
    if args.workload == "d3" and "d4" in legs:
        out["served"] = bench_d4(args)
    # the oracle from the timed run's final (steady) list
    out["cpu_baseline"] = (None if args.no_cpu else
                           cpu_baseline(cfg, keys, re, im, sc, args.cpu_seconds,
                                        args.cpu_cores))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
