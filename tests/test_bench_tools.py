"""bench.py's measurement helpers on synthetic inputs (no GPU): the source hash
that ties counter records to the kernels, the per-kernel summary of a
rocprofv3 kernel trace, and the counter summary that turns FETCH_SIZE /
WRITE_SIZE into HBM bytes with the probe's scale factors."""
import csv
import json
import os

import bench


def _sources():
    d = os.path.join(bench.ROOT, "paper_1802_05931_amd", "csrc")
    return {f: open(os.path.join(d, f)).read()
            for f in ("kernels.hpp", "model.hpp", "sampling.hpp", "ddqmc.hip")}


def test_source_hash_ignores_comments_but_not_code():
    src = _sources()
    h = bench.kernel_source_hash(src)
    assert h == bench.kernel_source_hash()
    commented = dict(src, **{"kernels.hpp": "// a new comment\n" + src["kernels.hpp"] +
                             "\n/* and a block\n comment */\n"})
    assert bench.kernel_source_hash(commented) == h
    changed = dict(src, **{"kernels.hpp": src["kernels.hpp"].replace(
        "constexpr int NT = 256;", "constexpr int NT = 128;")})
    assert changed["kernels.hpp"] != src["kernels.hpp"]
    assert bench.kernel_source_hash(changed) != h


def _write_trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, t0, t1 in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t1})


def test_trace_summary_counts_the_last_steps(tmp_path, capsys):
    # three steps, each: scan 10 us, loud 30 us, finalize 5 us (ns timestamps)
    rows, t = [], 0
    for _ in range(3):
        for name, dur in (("void ddqmc::k_spawn_scan<unsigned int>(...)", 10_000),
                          ("void ddqmc::k_spawn_loud<unsigned int>(...)", 30_000),
                          ("ddqmc::k_finalize(...)", 5_000)):
            rows.append((name, t, t + dur))
            t += dur + 1_000
    _write_trace(tmp_path / "x_kernel_trace.csv", rows)
    bench.trace_summary(str(tmp_path), 2)
    out = capsys.readouterr().out
    # the last two steps start after the first step's finalize
    assert "the last 2 steps, 6 dispatches" in out
    loud = [line for line in out.splitlines() if line.startswith("| k_spawn_loud")][0]
    cells = [c.strip() for c in loud.strip("|").split("|")]
    assert cells[1] == "2" and float(cells[3]) == 30.0 and float(cells[6]) == 30.0


def _write_counters(path, counter, values):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in values:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_counter_summary_scales_by_the_probe(tmp_path, monkeypatch, capsys):
    fetch, write = tmp_path / "fetch", tmp_path / "write"
    fetch.mkdir()
    write.mkdir()
    probe = "void at::native::elementwise_kernel<...>(...)"
    merge = "void ddqmc::k_merge<unsigned int, true>(...)"
    # the probe moves 1 MiB each way; FETCH_SIZE reports half of its reads
    _write_counters(fetch / "a_counter_collection.csv", "FETCH_SIZE",
                    [(probe, 512.0), (merge, 1000.0), (merge, 1000.0)])
    _write_counters(write / "a_counter_collection.csv", "WRITE_SIZE",
                    [(probe, 1024.0), (merge, 300.0), (merge, 300.0)])
    profiles = tmp_path / "profiles"
    profiles.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None: "feedfacefeedface")
    bench.counter_summary(str(fetch), str(write), 1, "t")
    out = capsys.readouterr().out
    assert "scale factors are 2.0000 (fetch) and 1.0000 (write)" in out
    rec = json.load(open(profiles / "k_merge_write_t_traffic.json"))
    # (1000 KiB x 2 + 300 KiB x 1) per dispatch
    assert abs(rec["bytes_per_launch"] - 2300 * 1024) < 1.0
    assert rec["source_hash"] == "feedfacefeedface"


def test_counter_records_apply_only_to_a_like_state(tmp_path, monkeypatch):
    """A counter record carries the mean list entries and spawn records of the
    run it was taken on; bench.py uses it only for a live run within 10% of
    both, and on the same kernel sources."""
    profiles = tmp_path / "profiles"
    profiles.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None: "feedfacefeedface")
    rec = {"bytes_per_launch": 2.5e8, "source_hash": "feedfacefeedface",
           "mean_entries": 1.08e7, "mean_spawn_records": 1.2e6}
    with open(profiles / "k_merge_write_d3_traffic.json", "w") as f:
        json.dump(rec, f)
    steady = dict(mean_entries=1.1e7, mean_spawn_records=1.25e6)
    assert bench.traffic_from_profile("k_merge_write", "d3", steady) == 2.5e8
    transient = dict(mean_entries=1394.0, mean_spawn_records=902.0)
    assert bench.traffic_from_profile("k_merge_write", "d3", transient) is None
    assert bench.traffic_from_profile("k_merge_write", "d3",
                                      dict(steady, mean_spawn_records=1.5e6)) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None: "0000000000000000")
    assert bench.traffic_from_profile("k_merge_write", "d3", steady) is None
    # a record without the state fields is never used
    monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None: "feedfacefeedface")
    with open(profiles / "k_spawn_loud_d3_valu.json", "w") as f:
        json.dump({"valu_per_launch": 6.9e7, "source_hash": "feedfacefeedface"}, f)
    assert bench.valu_from_profile("k_spawn_loud", "d3", steady) is None


class _FakeSolve:
    """Stands in for a handle: the list grows towards a steady size."""

    def __init__(self, final, rate):
        self.final, self.rate, self.n, self.steps = final, rate, 1.0, 0

    def step(self, k):
        for _ in range(k):
            self.n += (self.final - self.n) * self.rate
        self.steps += k

    def list_size(self):
        return int(self.n)


def test_equilibration_waits_for_a_steady_list():
    g = _FakeSolve(1e7, 3e-4)
    steps, steady, sizes = bench.equilibrate(g, log=lambda m: None)
    assert steady and steps >= bench.EQUIL_MIN and steps % bench.EQUIL_CHUNK == 0
    # the last two chunks changed the list by less than 1%, the two before by more
    assert abs(sizes[-1] - sizes[-3]) <= 0.01 * sizes[-1]
    assert abs(sizes[-2] - sizes[-4]) > 0.01 * sizes[-2]
    assert sizes[-1] > 0.95e7
    # a list already steady still takes the minimum number of steps
    g = _FakeSolve(1.0, 0.0)
    steps, steady, _ = bench.equilibrate(g, log=lambda m: None)
    assert steady and steps == bench.EQUIL_MIN


def test_counter_summary_by_request_size(tmp_path, monkeypatch, capsys):
    """With the request-size run, a kernel's read bytes are 32, 64 and 128
    bytes per request of each size; the record carries them beside the
    probe-scaled figure, and the kernel of several tile shapes that moved the
    most bytes is the one recorded."""
    dirs = {k: tmp_path / k for k in ("fetch", "write", "valu", "req")}
    for d in dirs.values():
        d.mkdir()
    probe = "void at::native::elementwise_kernel<...>(...)"
    m8 = "void ddqmc::k_merge<unsigned int, true, 8>(...)"
    m4 = "void ddqmc::k_merge<unsigned int, true, 4>(...)"
    _write_counters(dirs["fetch"] / "a_counter_collection.csv", "FETCH_SIZE",
                    [(probe, 512.0), (m8, 1000.0), (m4, 10.0)])
    _write_counters(dirs["write"] / "a_counter_collection.csv", "WRITE_SIZE",
                    [(probe, 1024.0), (m8, 300.0), (m4, 3.0)])
    _write_counters(dirs["valu"] / "a_counter_collection.csv", "SQ_INSTS_VALU", [(m8, 5.0)])
    with open(dirs["req"] / "a_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, c32, c64, c128 in ((probe, 0, 0, 8192), (m8, 1000, 4000, 2000),
                                     (m4, 10, 10, 10)):
            for b, c in (("32B", c32), ("64B", c64), ("128B", c128)):
                w.writerow({"Kernel_Name": name, "Counter_Name": f"TCC_EA0_RDREQ_{b}_sum",
                            "Counter_Value": c})
    profiles = tmp_path / "profiles"
    profiles.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda texts=None: "feedfacefeedface")
    bench.counter_summary(str(dirs["fetch"]), str(dirs["write"]), 1, "t", str(dirs["valu"]),
                          None, str(dirs["req"]))
    out = capsys.readouterr().out
    assert "by request sizes the probe read 1.0 MiB" in out
    rec = json.load(open(profiles / "k_merge_write_t_traffic.json"))
    assert rec["kernel"] == "k_merge<unsigned int, true, 8>"
    assert abs(rec["bytes_per_launch"] - 2300 * 1024) < 1.0
    reads = 32 * 1000 + 64 * 4000 + 128 * 2000
    assert abs(rec["bytes_per_launch_by_request_size"] - (reads + 300 * 1024)) < 1.0


def test_oracle_baseline_on_one_core_and_on_several():
    """The oracle baseline from a list and its scalars: one core in-process,
    then the aggregate of two pinned worker processes with seeds of their own."""
    import workloads
    from oracle import orc
    orc.build(force=False)
    cfg = dict(workloads.D1)
    o = orc.Oracle(**cfg)
    o.step(200)
    keys, re, im = o.get_list()
    sc = o.scalars()
    o.close()
    out = bench.cpu_baseline(cfg, keys, re, im, sc, budget_s=0.3, workers=2)
    assert out["kind"] == "oracle" and out["cores"] == 1
    assert out["value"] > 0 and out["entry_updates_per_s"] > 0
    assert out["host"]["nproc"] >= 1 and out["host"]["usable_cpus"] >= 1
    agg = out["all_cores"]
    assert agg["cores"] == 2 and agg["value"] > 0 and agg["entry_updates_per_s"] > 0
    assert "seeds 1..2" in agg["sample"]
    assert "all_cores" not in bench.cpu_baseline(cfg, keys, re, im, sc, budget_s=0.1,
                                                 workers=1)
