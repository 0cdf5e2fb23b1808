"""Benchmark of the Moss hot path on one MI355X.

Headline (`value`): the batched configuration C4.  256 estimation requests (k in {4, 5},
budgets log-uniform in [1e4, 1e7], 3.46e8 samples in all) over 32 resident Chung-Lu
graphs (m log-uniform in [1e3, 5e6]) run as one batched launch: a hipGraph-replayed
persistent kernel over a tile list, plus grouped launches for the large items on the
larger graphs, with the tile size and occupancy picked by the library's autotuner.
A step is one such launch over all 256 requests (the graphs' tables are built before the
timed steps: the graphs are resident); value = samples per second of wall time.

The same JSON line also carries:
  batched       the same requests with one moss_estimate call per request (the plain
                form), the batched launch with the default tuning, and whether every
                request's result is identical in all three
  plain         C2 (4-node, n=1e5, m=1e6, 1e7 samples) and C3 (5-node, n=1e6, m=1e7,
                1e8 samples): a step = create over the device CSR + validate + build the
                tables + sample and classify + finals; per-motif estimates, Theorem 3/10
                standard errors and, for C2, relative errors against exact counts
  accuracy5     C1 at k=5 with 1e7 samples against the exact 5-node counts (ESU)
  serving       C5: Poisson arrivals at 500 req/s over 64 resident graphs (up to n=4e6,
                m=3.5e7), k in {4,5}, budgets log-uniform in [1e4, 1e8], a finite table
                memory budget (evictions), p50/p99 latency, sustained against offered
                samples/s, and served results compared with the same requests alone
  roofline      of the headline launch (and per plain workload): device bytes moved past
                the L2s and L2 requests per launch, from the committed rocprofv3 counter
                summaries of the same command (profiles/counters_<workload>.md, used only
                when taken on the current kernel sources), over the launch's device time
                measured live with HIP events on its stream; frac is the larger of
                fabric bytes/s / 8 TB/s and L2 requests/s / (128 channels x L2 clock)
  gather        the random-gather ceiling: chains of dependent 8-byte loads, several
                chains per lane, over a buffer the size of the C3 samplers' footprint
                (libmoss_probe.so)
  cpu_baseline  the oracle (plain C) on the host cores: a bounded sample of the C4
                requests (each request's first 2^15 samples per sampler), all cores and
                one core, median of 5 runs, CPU model stated

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
       python bench.py --only c4-step|c2-step|c3-step --steps 2 --warmup 1   (counter runs)
       python bench.py --summarize-counters DIR [DIR ...] --workload C4 --launches 3
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import platform
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "graphlet samples/sec (4-,5-node) batched vs plain; serving p50/p99 latency"
PEAK_HBM_GBS = 8000.0
L2_CHANNELS = 128           # 16 per XCD x 8 XCDs
L2_CLOCK_HZ_NOMINAL = 2.4e9  # peak engine clock; the counter summaries measure the actual one

WORKLOAD_TEXT = {
    "C1": "plain 4-node MOSS-4, Chung-Lu n=2e3 m=1e4 beta=2.5 dmax=200, 1e5 samples, seed 1",
    "C2": "plain 4-node MOSS-4, Chung-Lu n=1e5 m=1e6 beta=2.2 dmax=3e3, 1e7 samples, seed 1",
    "C3": "plain 5-node MOSS-5 (T-5 + Path-5), Chung-Lu n=1e6 m=1e7 beta=2.1 dmax=2e4, 1e8 samples, seed 1",
    "C4": "batched: 256 requests (k in {4,5}, budgets log-uniform 1e4..1e7) over 32 resident Chung-Lu graphs "
          "(m log-uniform 1e3..5e6), one persistent hipGraph launch with autotuned tiles",
    "C5": "serving: Poisson 500 req/s over 64 resident Chung-Lu graphs (m 1e3..3.5e7, largest n=4e6 beta=2.0), "
          "k in {4,5}, budgets log-uniform 1e4..1e8, memory-based admission",
}

# kernels that run between the HIP events bracketing a sampling launch (moss_estimate's
# grouping passes and sampling kernels; the batched launch's clear, persistent kernel
# and grouped launches)
LAUNCH_KERNELS = ("k_sort_count", "k_sort_runsum", "k_sort_runscan", "k_sort_place", "k_sort_scatter",
                  "k_sample_sorted", "k_sample<", "k_batch", "k_fill_u64", "k_fill_u32")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", default="", help="comma list of c4,c2,c3,c5,acc5,probe,cpu,c2min,c3min; or c4-step, "
                                               "c2-step, c3-step, c2min-step, c3min-step (just the timed steps, for "
                                               "counter runs)")
    ap.add_argument("--tuning", default="", metavar="T,B,G,F[,W]",
                    help="c4-step: the batched launch's tiles, blocks per CU, grouping thresholds (2^G samples, "
                         "F MB) and sorted window W as the full run's autotuner picked them (default: the "
                         "library's)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget-gib", type=float, default=4.0, help="table memory budget of the server")
    ap.add_argument("--serve-chunk", type=int, default=0, help="server: samples per request per iteration (0: 2^25)")
    ap.add_argument("--serve-iteration", type=int, default=0, help="server: samples per iteration (0: 2^25)")
    ap.add_argument("--serve-express", type=int, default=0,
                    help="server: requests of at most this many samples take the express path (0: 2^22; "
                         "negative: none)")
    ap.add_argument("--probe-only", type=int, default=0, metavar="BYTES",
                    help="only run the gather probe over a buffer of BYTES (for its counters)")
    ap.add_argument("--probe-chains", type=int, default=8)
    ap.add_argument("--probe-waves", type=int, default=16)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times)")
    ap.add_argument("--summarize-counters", nargs="+", default=None, metavar="DIR",
                    help="print the counter summary of rocprofv3 output directories (no GPU)")
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--launches", type=int, default=3, help="launches of the workload in the counter runs")
    ap.add_argument("--source-sha", default=None,
                    help="kernel_source_sha the counter runs printed (default: the current sources')")
    ap.add_argument("--kernels", default=",".join(LAUNCH_KERNELS),
                    help="kernel name parts the counter summary keeps (comma list)")
    return ap.parse_args()


# ---------------------------------------------------------------------------------------
# host facts
def host_cores() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def kernel_source_sha() -> str:
    """Hash of the device sources (kernels and the device helpers they include)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "device.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1509_08089_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------------------
# rocprofv3 counter summaries
def _counter_rows(dirs):
    for d in dirs:
        for p in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(p, newline="") as f:
                yield from csv.DictReader(f)


def _trace_rows(dirs):
    for d in dirs:
        for p in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
            with open(p, newline="") as f:
                yield from csv.DictReader(f)


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").split("(")[0]
    return name.replace("moss::", "").replace("void ", "").strip()


def summarize_counters(dirs, workload: str, launches: int, kernels=LAUNCH_KERNELS, source_sha=None) -> str:
    """Per-kernel sums of the counters in rocprofv3 --pmc output directories (one pass per
    directory, each a run of `launches` launches of the workload), restricted to the
    kernels of the sampling launch, divided per launch; plus kernel durations from any
    kernel-trace output among the directories."""
    per = {}      # kernel -> counter -> sum
    disp = {}     # (kernel, counter) -> dispatch ids
    for row in _counter_rows(dirs):
        kn = _short(row.get("Kernel_Name", ""))
        if not any(_short(k) in kn for k in kernels):
            continue
        cn = row.get("Counter_Name", "")
        val = float(row.get("Counter_Value", 0) or 0)
        per.setdefault(kn, {}).setdefault(cn, 0.0)
        per[kn][cn] += val
        disp.setdefault((kn, cn), set()).add(row.get("Dispatch_Id", row.get("Correlation_Id", "")))
    dur = {}      # kernel -> durations (us) over every traced run
    traced = 0    # runs with a kernel trace
    for d in dirs:
        rows = list(_trace_rows([d]))
        traced += bool(rows)
        for row in rows:
            kn = _short(row.get("Kernel_Name", ""))
            if kn in per or any(_short(k) in kn for k in kernels):
                try:
                    us = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
                except (KeyError, ValueError):
                    continue
                dur.setdefault(kn, []).append(us)
    tot = {}
    for kn, cs in per.items():
        for cn, v in cs.items():
            tot[cn] = tot.get(cn, 0.0) + v / launches

    def g(cn):
        return tot.get(cn, 0.0)

    read_b = 32 * g("TCC_EA0_RDREQ_32B_sum") + 64 * g("TCC_EA0_RDREQ_64B_sum") + 128 * g("TCC_EA0_RDREQ_128B_sum")
    other = g("TCC_EA0_RDREQ_sum") - g("TCC_EA0_RDREQ_32B_sum") - g("TCC_EA0_RDREQ_64B_sum") - \
        g("TCC_EA0_RDREQ_128B_sum")
    write_b = 32 * (g("TCC_EA0_WRREQ_sum") - g("TCC_EA0_WRREQ_64B_sum")) + 64 * g("TCC_EA0_WRREQ_64B_sum")
    lines = [f"kernel_source_sha: {source_sha or kernel_source_sha()}", f"workload: {workload}",
             f"launches_in_run: {launches}"]
    kern_us = sum(sum(v) for v in dur.values()) / (launches * traced) if traced else 0.0
    lines.append(f"launch_kernel_us: {kern_us:.3f}")
    for cn in sorted(tot):
        lines.append(f"per_launch {cn}: {tot[cn]:.6e}")
    lines.append(f"read_bytes_per_launch: {read_b:.6e}")
    lines.append(f"rdreq_unsized_per_launch: {other:.6e}")
    lines.append(f"write_bytes_per_launch: {write_b:.6e}")
    lines.append(f"fabric_bytes_per_launch: {read_b + write_b:.6e}")
    lines.append(f"ea_rdreq_per_launch: {g('TCC_EA0_RDREQ_sum'):.6e}")
    lines.append(f"tcc_req_per_launch: {g('TCC_REQ_sum'):.6e}")
    if g("TCC_CYCLE_sum") and kern_us:
        lines.append(f"l2_clock_hz: {g('TCC_CYCLE_sum') / L2_CHANNELS / (kern_us * 1e-6):.6e}")
    if g("TCC_BUSY_sum") and g("TCC_CYCLE_sum"):
        lines.append(f"l2_busy_frac: {g('TCC_BUSY_sum') / g('TCC_CYCLE_sum'):.4f}")
    if g("TCC_HIT_sum") + g("TCC_MISS_sum"):
        lines.append(f"l2_hit_rate: {g('TCC_HIT_sum') / (g('TCC_HIT_sum') + g('TCC_MISS_sum')):.4f}")
    lines.append("")
    lines.append("| kernel | dispatches/launch | avg us | " + " | ".join(sorted({c for cs in per.values() for c in cs}))
                 + " |")
    lines.append("|---" * (3 + len({c for cs in per.values() for c in cs})) + "|")
    for kn in sorted(per, key=lambda k: -sum(dur.get(k, [0]))):
        cs = per[kn]
        nd = len(dur[kn]) / (launches * traced) if kn in dur else float("nan")
        avg = statistics.mean(dur[kn]) if kn in dur else float("nan")
        lines.append(f"| `{kn}` | {nd:g} | {avg:.1f} | " +
                     " | ".join(f"{cs.get(c, 0.0) / launches:.4e}" for c in sorted({c for x in per.values() for c in x}))
                     + " |")
    return "\n".join(lines)


def read_counter_summary(workload: str):
    """The machine-readable lines of profiles/counters_<workload>.md, if that summary was
    taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"counters_{workload}.md")
    if not os.path.exists(p):
        return None
    out = {}
    for line in open(p):
        m = re.match(r"^([a-z0-9_]+(?: [A-Za-z0-9_]+)?):\s*([0-9a-fA-F.eE+-]+)\s*$", line.strip())
        if m:
            out[m.group(1)] = m.group(2)
    if out.get("kernel_source_sha") != kernel_source_sha():
        return None
    return {k: (v if k == "kernel_source_sha" else float(v)) for k, v in out.items() if k != "workload"}


def roofline(workload: str, device_ms: float, alg_bytes: float | None, samples: float):
    """Fabric bytes and L2 requests of one launch (committed counter summary) over the
    launch's live device time; the binding one of the two sets frac."""
    c = read_counter_summary(workload)
    secs = device_ms / 1e3
    out = {"workload": workload, "launch_ms": device_ms, "alg_bytes_per_launch": alg_bytes,
           "alg_gbs": alg_bytes / secs / 1e9 if alg_bytes else None,
           "launch_samples_per_s": samples / secs}
    if not c:
        out.update({"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                    "traffic": None, "note": "no counter summary taken on the current kernel sources"})
        return out
    fabric = c["fabric_bytes_per_launch"]
    fab_gbs = fabric / secs / 1e9
    clock = c.get("l2_clock_hz", L2_CLOCK_HZ_NOMINAL)
    req_s = c["tcc_req_per_launch"] / secs
    l2_cap = L2_CHANNELS * clock
    fab = {"achieved": fab_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": fab_gbs / PEAK_HBM_GBS,
           "bytes_per_launch": fabric, "read_bytes": c["read_bytes_per_launch"],
           "write_bytes": c["write_bytes_per_launch"], "bytes_per_sample": fabric / samples}
    l2 = {"achieved": req_s / 1e9, "peak": l2_cap / 1e9, "unit": "Greq/s", "frac": req_s / l2_cap,
          "requests_per_launch": c["tcc_req_per_launch"], "requests_per_sample": c["tcc_req_per_launch"] / samples,
          "l2_clock_hz": clock, "hit_rate": c.get("l2_hit_rate"), "busy_frac": c.get("l2_busy_frac")}
    if fab["frac"] >= l2["frac"]:
        out.update({"bound": "hbm", "achieved": fab_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": fab["frac"]})
    else:
        out.update({"bound": "l2", "achieved": l2["achieved"], "peak": l2["peak"], "unit": "Greq/s",
                    "frac": l2["frac"]})
    out.update({"traffic": fabric, "fabric": fab, "l2": l2,
                "counter_launch_kernel_us": c.get("launch_kernel_us")})
    return out


# ---------------------------------------------------------------------------------------
# measurements
def copy_calibration(nbytes: int) -> int:
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reads_per_dispatch": nbytes, "writes_per_dispatch": nbytes}))
    return 0


def gather_ceiling(footprint_bytes: int, waves=(8, 16, 32), chains=(1, 4, 8), loads=1 << 27):
    """Chains of dependent random 8-byte loads over a buffer of the given size: loads/s
    for each occupancy and number of chains per lane, and the best."""
    import torch
    from paper_1509_08089_amd import probe
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    buf = torch.empty(max(1, footprint_bytes // 8), dtype=torch.int64, device="cuda")
    probe.moss_probe_fill(buf, 1)
    sweep = {}
    for w in waves:
        for c in chains:
            blocks = cus * w // 4  # 256-lane blocks of four waves
            out = torch.empty(blocks * 256, dtype=torch.int64, device="cuda")
            steps = max(16, loads // (blocks * 256 * c))
            probe.moss_probe_gather(buf, blocks, steps, out, c)  # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                probe.moss_probe_gather(buf, blocks, steps, out, c)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            sweep[f"{w}w{c}c"] = blocks * 256 * steps * c / (ms / 1e3)
    best = max(sweep, key=sweep.get)
    return {"footprint_bytes": int(buf.numel() * 8), "loads_per_s": sweep[best], "best": best,
            "sweep_loads_per_s": sweep}


# buffer sizes of the gather probe: inside one CU's vector L1 (32 KB), inside one XCD's
# L2 (4 MB), past the eight L2s (32 MB in all) but inside the 256 MB MALL, and the C3
# samplers' footprint (past the MALL)
PROBE_LEVELS = {"l1": 16 << 10, "l2": 2 << 20, "mall": 48 << 20}


def gather_levels(line, plain):
    """The random-gather ceilings of each level of the memory hierarchy (dependent
    8-byte loads at random places, several chains per lane, best occupancy), and each
    sampling launch's rate at that level against them: L2 requests (TCC_REQ) against the
    L2-resident probe (whose loads each make one L2 request), read requests past the L2s
    (TCC_EA0_RDREQ) against the best probe whose buffer exceeds the L2s.  The L1-resident
    probe and the kernels' vector-L1 line accesses are reported beside them (a wave's
    loads into a 16 KB buffer share lines, so that probe's loads are not line accesses)."""
    sizes = dict(PROBE_LEVELS, hbm=plain["C3"]["sampling_bytes"] if "C3" in plain else 665_683_712)
    out = {"levels": {}}
    for lvl, nbytes in sizes.items():
        out["levels"][lvl] = gather_ceiling(nbytes, waves=(16, 32), chains=(1, 8))
    fabric_ceiling = max(out["levels"]["mall"]["loads_per_s"], out["levels"]["hbm"]["loads_per_s"])
    out["fabric_lines_per_s"] = fabric_ceiling
    launches = {name: p["sampling_launch_ms"] for name, p in plain.items()}
    if "batched" in line:
        launches["C4"] = line["batched"]["device_ms"]
    for name, ms in launches.items():
        c = read_counter_summary(name)
        if not c:
            continue
        secs = ms / 1e3
        rates = {"tcp_accesses_per_s": c.get("per_launch TCP_TOTAL_CACHE_ACCESSES_sum", 0.0) / secs,
                 "l2_requests_per_s": c["tcc_req_per_launch"] / secs,
                 "fabric_reads_per_s": c["ea_rdreq_per_launch"] / secs}
        rates["l2_frac"] = rates["l2_requests_per_s"] / out["levels"]["l2"]["loads_per_s"]
        rates["fabric_frac"] = rates["fabric_reads_per_s"] / fabric_ceiling
        out[name] = rates
    if "C4" in out:
        out["frac"] = max(out["C4"]["l2_frac"], out["C4"]["fabric_frac"])
    return out


def exact_counts(workload: str, sha: str, key: str):
    p = os.path.join(ROOT, "tests", "golden", f"exact_{workload.lower()}.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("graph_sha256") != sha:
        return None
    return d.get(key)


def line_counts():
    return json.load(open(os.path.join(ROOT, "tests", "golden", "line_counts.json")))


def errors(r, exact):
    est = [float(x) for x in r.estimate_np]
    out = {"estimates": est,
           "stderr_rel": [float(math.sqrt(max(v, 0.0)) / e) if e > 0 else None for v, e in zip(r.variance_np, est)]}
    if exact is not None:
        out["exact"] = exact
        out["rel_error"] = [abs(e - x) / x if x else None for e, x in zip(est, exact)]
        out["stderr_rel_vs_exact"] = [float(math.sqrt(max(v, 0.0)) / x) if x else None
                                      for v, x in zip(r.variance_np, exact)]
    return out


def run_c4(moss, gg, args, step_only=False):
    import numpy as np
    import torch
    specs, reqs = gg.batch_workload()
    log(f"[bench] C4: generating {len(specs)} graphs on the device")
    graphs = [moss.Graph.from_device(*s.build_device()) for s in specs]
    torch.cuda.synchronize()
    q = [(graphs[r.graph].h, r.k, r.samples, r.seed, 0) for r in reqs]
    total = sum(r.samples for r in reqs)
    t = time.perf_counter()
    for g in graphs:
        g.build_tables()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    log(f"[bench] C4: tables built ({build_s:.2f} s)")
    out = {"requests": len(q), "graphs": len(graphs), "samples": total, "table_build_s": build_s}
    if step_only and args.tuning:
        tile, bpc, gs, gf, win = ([int(x) for x in args.tuning.split(",")] + [0])[:5]
        moss.moss_set_tuning(tile, bpc, 0, 0, gs, gf, win)
        out["tuning"] = {"tile_samples": tile, "blocks_per_cu": bpc, "group_min_samples_log2": gs,
                         "group_min_footprint_mb": gf, "sort_window": win}
    if not step_only:
        best, tune_ms = moss.moss_autotune(q)
        out["tuning"] = {"tile_samples": best.tile_samples, "blocks_per_cu": best.blocks_per_cu,
                         "group_min_samples_log2": best.group_min_samples_log2,
                         "group_min_footprint_mb": best.group_min_footprint_mb, "sort_window": best.sort_window,
                         "autotune_best_ms": tune_ms}
        log(f"[bench] C4: autotuned ({best.tile_samples} samples per tile, {best.blocks_per_cu} blocks/CU, grouping "
            f"thresholds {best.group_min_samples_log2 or 'default'} / {best.group_min_footprint_mb or 'default'})")
    for i in range(args.warmup):
        moss.moss_estimate_batch(q)
        log(f"[bench] C4 warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [moss.moss_estimate_batch(q) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[bench] C4: {args.steps} timed steps done")
    ms = (t1 - t0) * 1e3 / args.steps
    dev_ms = sum(r[0].device_ms for r in runs) / len(runs)
    out.update({"ms_per_step": ms, "batched_samples_per_s": total / (ms / 1e3), "device_ms": dev_ms})
    if step_only:
        return out, runs[0]
    same = all(np.array_equal(a.hits_np, b.hits_np) for r in runs[1:] for a, b in zip(runs[0], r))

    def timed(fn, reps=3):  # median wall time of `reps` calls after one warm-up call
        res = fn()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            res = fn()
            ts.append(time.perf_counter() - t)
        return statistics.median(ts), res

    moss.moss_set_tuning(0, 0, 0)
    t_default, got_default = timed(lambda: moss.moss_estimate_batch(q))
    t_plain, alone = timed(lambda: [moss.moss_estimate(*x) for x in q])
    same = same and all(np.array_equal(a.hits_np, b.hits_np) and np.array_equal(a.estimate_np, b.estimate_np)
                        for a, b in zip(alone, runs[0]))
    same = same and all(np.array_equal(a.hits_np, b.hits_np) for a, b in zip(alone, got_default))
    log("[bench] C4: one launch per request timed")
    out.update({"plain_samples_per_s": total / t_plain, "default_tuning_samples_per_s": total / t_default,
                "speedup_vs_plain": t_plain / (ms / 1e3), "identical_results": bool(same)})
    return out, runs[0]


def plain_steps(moss, gg, args, name, with_min=False):
    """Whole-path steps of a plain workload: create over the device CSR, build the tables,
    estimate, destroy.  With with_min, the graph of `name` with MOSS-4 and MOSS-4Min on
    half of 1e7 samples each (their rank tables built in the step) and the 4-node mix."""
    import numpy as np
    import torch
    cfg = dict(gg.CONFIGS[name])
    if with_min:
        cfg.update(k=4, samples=10_000_000)
    log(f"[bench] {name}: generating the graph")
    t = time.perf_counter()
    csr = cfg["graph"].build()
    log(f"[bench] {name}: graph ready ({time.perf_counter() - t:.1f} s)")
    k, K, seed = cfg["k"], cfg["samples"], cfg["seed"]
    flags = moss.MOSS_K4_MIN if with_min else 0
    mask = (moss.MOSS_TABLES_K4 | (moss.MOSS_TABLES_K4MIN if with_min else 0)) if k == 4 else moss.MOSS_TABLES_K5
    d_rp = torch.from_numpy(csr.row_ptr).cuda()
    d_col = torch.from_numpy(csr.col).cuda()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step():
        h = moss.moss_graph_create_device(csr.n, csr.nnz, d_rp, d_col, 0, stream)
        try:
            moss.moss_build_tables(h, mask)
            return moss.moss_estimate(h, k, K, seed, flags)
        finally:
            moss.moss_graph_destroy(h)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[bench] {name}: {args.steps} timed steps done")
    ms = (t1 - t0) * 1e3 / args.steps
    for r in results[1:]:
        assert np.array_equal(r.hits_np, results[0].hits_np)
    r0 = results[0]
    dev_ms = sum(r.device_ms for r in results) / len(results)
    lc = line_counts()[name]
    if with_min:
        alg = 64.0 * (r0.K[0] * lc["moss4"] + r0.K[1] * lc["moss4min"]) if "moss4min" in lc else None
    elif k == 4:
        alg = 64.0 * K * lc["moss4"]
    else:
        alg = 64.0 * (r0.K[0] * lc["t5"] + r0.K[1] * lc["path5"])
    text = (f"{name} graph with MOSS-4 + MOSS-4Min (5e6 + 5e6 samples, rank tables built in the step), 4-node "
            f"mix, seed 1" if with_min else f"{name}: {WORKLOAD_TEXT[name]}")
    out = {"workload": text, "n": csr.n, "m": csr.m, "k": k, "samples": K,
           "graph_sha256": csr.sha256()[:16], "ms_per_step": ms, "samples_per_s": K / (ms / 1e3),
           "sampling_launch_ms": dev_ms, "lines_per_sample": {s: lc[s] for s in ("moss4", "t5", "path5") if s in lc}}
    out["roofline"] = roofline(name + ("MIN" if with_min else ""), dev_ms, alg, K)
    out.update(errors(r0, exact_counts(name, csr.sha256(), "n4" if k == 4 else "eta5")))
    info_h = moss.moss_graph_create_device(csr.n, csr.nnz, d_rp, d_col, 0, stream)
    try:
        moss.moss_build_tables(info_h, mask)
        out["sampling_bytes"] = int(moss.moss_graph_get_info(info_h).sampling_bytes)
    finally:
        moss.moss_graph_destroy(info_h)
    if not with_min:
        out["table_build_ms"] = table_builds(moss, csr, d_rp, d_col, stream)
    return out, csr


def table_builds(moss, csr, d_rp, d_col, stream, reps=5):
    """Wall time of moss_build_tables on a freshly created graph (median of `reps` after
    one warm-up each), per table set; "moss4min_part" = (4-node + MOSS-4Min) - 4-node."""
    import torch
    sets = {"k4": moss.MOSS_TABLES_K4, "k4+moss4min": moss.MOSS_TABLES_K4 | moss.MOSS_TABLES_K4MIN,
            "k5": moss.MOSS_TABLES_K5}
    out = {}
    for label, mask in sets.items():
        times = []
        for i in range(reps + 1):
            h = moss.moss_graph_create_device(csr.n, csr.nnz, d_rp, d_col, 0, stream)
            try:
                torch.cuda.synchronize()
                t = time.perf_counter()
                moss.moss_build_tables(h, mask)
                torch.cuda.synchronize()
                if i:
                    times.append((time.perf_counter() - t) * 1e3)
            finally:
                moss.moss_graph_destroy(h)
        out[label] = sorted(times)[len(times) // 2]
    out["moss4min_part"] = out["k4+moss4min"] - out["k4"]
    return out


def accuracy5(moss, gg):
    """C1 graph, k=5, 1e7 samples, against the exact 5-node counts (ESU)."""
    csr = gg.config_graph("C1")
    G = moss.Graph(csr)
    r = G.estimate(5, 10_000_000, 1)
    out = {"workload": "C1 graph (Chung-Lu n=2e3 m=1e4 beta=2.5 dmax=200), k=5, 1e7 samples, seed 1",
           "device_ms": r.device_ms}
    out.update(errors(r, exact_counts("C1", csr.sha256(), "eta5")))
    G.close()
    return out


def run_serving(moss, gg, args):
    import numpy as np
    import torch
    specs, reqs = gg.serving_workload(n_requests=args.serve_requests)
    log(f"[bench] C5: generating {len(specs)} graphs on the device")
    graphs = [moss.Graph.from_device(*s.build_device()) for s in specs]
    torch.cuda.synchronize()
    log("[bench] C5: graphs ready")
    budget = int(args.serve_budget_gib * (1 << 30))
    srv = moss.moss_server_create(budget, 256, args.serve_chunk, iteration_samples=args.serve_iteration,
                                  express_samples=max(args.serve_express, 0), express=args.serve_express >= 0)
    results = {}
    try:
        ids = [moss.moss_server_add_graph(srv, g.h) for g in graphs]
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            now = time.perf_counter() - t0
            if r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            tickets.append(moss.moss_server_submit(srv, ids[r.graph], r.k, r.samples, r.seed))
        check = set(range(0, len(reqs), max(1, len(reqs) // 40)))
        for i, tk in enumerate(tickets):
            res = moss.moss_server_wait(srv, tk, -1)
            if i in check:
                results[i] = res
        wall = time.perf_counter() - t0
        st = moss.moss_server_stats_get(srv)
    finally:
        moss.moss_server_destroy(srv)
    log(f"[bench] C5: {len(reqs)} requests served ({wall:.1f} s)")
    same = True
    for i, res in results.items():
        r = reqs[i]
        alone = moss.moss_estimate(graphs[r.graph].h, r.k, r.samples, r.seed, 0)
        same = same and np.array_equal(alone.hits_np, res.hits_np) and np.array_equal(alone.estimate_np,
                                                                                      res.estimate_np)
    offered = sum(r.samples for r in reqs) / reqs[-1].arrival_s
    return {"workload": f"C5: {WORKLOAD_TEXT['C5']}", "requests": len(reqs), "graphs": len(graphs),
            "edges": int(sum(s.m for s in specs)), "rate_req_s": len(reqs) / reqs[-1].arrival_s,
            "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "samples_per_s": st.samples_per_s,
            "offered_samples_per_s": offered, "wall_s": wall, "iterations": st.iterations,
            "mem_budget_bytes": budget, "evictions": int(st.evictions),
            "chunk_samples": args.serve_chunk or 1 << 25, "iteration_samples": args.serve_iteration or 1 << 25,
            "express_samples": (args.serve_express or 1 << 22) if args.serve_express >= 0 else None,
            "express_launches": int(st.express_launches),
            "checked_against_alone": len(results), "identical_results": bool(same)}


def cpu_baseline(moss, gg, cap=1 << 15, runs=5):
    """The oracle on a bounded sample of the C4 requests: each request's samples
    [0, min(K_l, cap)) of each of its samplers, graph by graph (the oracle's table build
    is not timed), all host cores and one core, median of `runs` runs."""
    import numpy as np
    import oracle
    from graphgen.csr import CSR
    specs, reqs = gg.batch_workload()
    cores = host_cores()
    by_graph = {}
    for r in reqs:
        by_graph.setdefault(r.graph, []).append(r)
    t_all = [0.0] * runs
    t_one = [0.0] * runs
    done = 0
    build_s = 0.0
    for gi, rs in sorted(by_graph.items()):
        rp, col = specs[gi].build_device()
        csr = CSR(rp.cpu().numpy(), col.cpu().numpy(), f"C4 graph {gi}")
        del rp, col
        t = time.perf_counter()
        og = oracle.Graph(csr)
        build_s += time.perf_counter() - t
        tot = og.totals()
        jobs = []
        for r in rs:
            if r.k == 4:
                if tot["gamma"]:
                    jobs.append((oracle.MOSS4, r.seed, min(r.samples, cap)))
            else:
                k1, k2 = (r.samples + 1) // 2, r.samples // 2
                if tot["gamma1"]:
                    jobs.append((oracle.T5, r.seed, min(k1, cap)))
                if tot["gamma2"]:
                    jobs.append((oracle.PATH5, r.seed, min(k2, cap)))
        done += sum(n for _, _, n in jobs)
        for i in range(runs):
            for threads, acc in ((cores, t_all), (1, t_one)):
                t = time.perf_counter()
                for sid, seed, n in jobs:
                    og.run(sid, seed, 0, n, threads)
                acc[i] += time.perf_counter() - t
        del og
    med_all, med_one = statistics.median(t_all), statistics.median(t_one)
    return {"value": done / med_all, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "single_core_samples_per_s": done / med_one, "cpu_model": cpu_model(),
            "sample": f"C4 requests, each request's first min(K_l, {cap}) samples of each of its samplers "
                      f"({done} samples over {len(by_graph)} graphs), {cores} threads over contiguous index "
                      f"ranges and 1 thread, median of {runs} runs each; the oracle's table build "
                      f"({build_s:.1f} s) not included",
            "runs_s_all_cores": t_all, "runs_s_one_core": t_one}


def main():
    args = parse()
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.workload, args.launches,
                                 tuple(k for k in args.kernels.split(",") if k), args.source_sha))
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sampler shards by sample "
                                   "ranges with one histogram all-reduce, which is not built here",
                          "n_gpus": args.gpus}))
        return 2
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.probe_only:
        print(json.dumps({"gather_probe": gather_ceiling(args.probe_only, waves=(args.probe_waves,),
                                                         chains=(args.probe_chains,))}), flush=True)
        return 0

    import torch

    import graphgen as gg
    from paper_1509_08089_amd import moss

    torch.cuda.init()
    only = set(x for x in args.only.split(",") if x)
    if only & {"c4-step", "c2-step", "c3-step", "c2min-step", "c3min-step"}:
        name = next(iter(only))
        if name == "c4-step":
            res, _ = run_c4(moss, gg, args, step_only=True)
        else:
            res, _ = plain_steps(moss, gg, args, name[:2].upper(), with_min="min" in name)
            res = {k: res[k] for k in ("ms_per_step", "samples_per_s", "sampling_launch_ms")}
        print(json.dumps({"step_only": name, "kernel_source_sha": kernel_source_sha(), **res}), flush=True)
        return 0
    parts = only or {"c4", "c2", "c3", "c5", "acc5", "probe", "cpu"}
    line = {"metric": METRIC, "value": None, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"C4: {WORKLOAD_TEXT['C4']}"}}
    if "c4" in parts:
        c4, _ = run_c4(moss, gg, args)
        line["value"] = c4["batched_samples_per_s"]
        line["ms_per_step"] = c4["ms_per_step"]
        line["config"].update({"requests": c4["requests"], "graphs": c4["graphs"], "samples": c4["samples"],
                               "step": "one batched launch over all 256 requests (tables resident)"})
        line["roofline"] = roofline("C4", c4["device_ms"], None, c4["samples"])
        line["batched"] = c4
    plain = {}
    for name in ("C2", "C3"):
        if name.lower() in parts:
            plain[name], _ = plain_steps(moss, gg, args, name)
    for name in ("C2", "C3"):  # MOSS-4 + MOSS-4Min on the plain graphs (only when asked)
        if name.lower() + "min" in parts:
            plain[name + "MIN"], _ = plain_steps(moss, gg, args, name, with_min=True)
    if plain:
        line["plain"] = plain
    if "acc5" in parts:
        line["accuracy5"] = accuracy5(moss, gg)
        log("[bench] C1 k=5 accuracy done")
    if "c5" in parts:
        line["serving"] = run_serving(moss, gg, args)
    if "probe" in parts:
        log("[bench] gather probe")
        line["gather"] = gather_levels(line, plain)
    if "cpu" in parts:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(moss, gg)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
