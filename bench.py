"""Benchmark of the Moss hot path on one MI355X.

A step is one pass of the whole path over the workload's graph, whose CSR is already
resident in HBM: create the graph handle over the device CSR (validation), build the
sampling tables (Section 4.1.3 initialization), draw and classify every sample
(Algorithm 1, or Algorithms 3 and 4), reduce the histograms and compute the FP64
finals.  The default workload is the plain 4-node configuration (Chung-Lu n=1e5,
m=1e6, 1e7 samples, seed 1).  value = samples drawn per second of wall time.
C2MIN is the same graph and budget with MOSS-4 and MOSS-4Min (Section 4.2) on half the
samples each, their rank tables built in the step, and the 4-node mix.

Also reported on the same JSON line:
  roofline      algorithmic bytes of the sampling kernel per launch (64 B per line
                read, line counts from tests/golden/line_counts.json) over its average
                duration from HIP events on the stream it runs on, against 8 TB/s
  cpu_baseline  the oracle's sampling loop timed on the host cores on a bounded
                prefix of the same sample stream
  gather        the dependent random-gather ceiling over a buffer of the samplers'
                footprint (libmoss_probe.so, best of several occupancies), and the
                kernel's vector-L1 line accesses per second (L1 accesses per sample from
                the committed counter summary) as a fraction of it
  batched       (--batched) 256 mixed requests over 32 graphs: one persistent launch
                vs one launch per request
  serving       (--serve) Poisson arrivals over many resident graphs: p50/p99 latency

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--workload C2|C3|C2MIN]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

WORKLOAD_TEXT = {
    "C1": "plain 4-node MOSS-4, Chung-Lu n=2e3 m=1e4 beta=2.5 dmax=200, 1e5 samples, seed 1",
    "C2": "plain 4-node MOSS-4, Chung-Lu n=1e5 m=1e6 beta=2.2 dmax=3e3, 1e7 samples, seed 1",
    "C3": "plain 5-node MOSS-5 (T-5 + Path-5), Chung-Lu n=1e6 m=1e7 beta=2.1 dmax=2e4, 1e8 samples, seed 1",
    "C2MIN": "4-node MOSS-4 + MOSS-4Min mix (5e6 + 5e6 samples), Chung-Lu n=1e5 m=1e6 beta=2.2 dmax=3e3, "
             "seed 1",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "C3", "C2MIN"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gather-probe", action="store_true")
    ap.add_argument("--probe-only", type=int, default=0, metavar="BYTES",
                    help="only run the gather probe over a buffer of BYTES (for its counters)")
    ap.add_argument("--batched", action="store_true")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times), to scale HBM counters")
    return ap.parse_args()


def copy_calibration(nbytes: int) -> int:
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reads_per_dispatch": nbytes, "writes_per_dispatch": nbytes}))
    return 0


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def kernel_source_sha() -> str:
    """Hash of the device sources (kernels and the device helpers they include)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "device.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1509_08089_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was taken
    on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(p):
        return None
    text = open(p).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_sha():
        return None
    return float(b.group(1))


def measured_l1_per_sample(kernel: str, workload: str):
    """Vector-L1 line accesses per sample of the sampling kernel, from the committed
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(p):
        return None
    text = open(p).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", text)
    b = re.search(r"l1_line_accesses_per_sample:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_sha():
        return None
    return float(b.group(1))


def gather_ceiling(footprint_bytes: int, waves_per_cu=(8, 16, 20, 32), loads=1 << 27):
    """Dependent random gathers over a buffer of the sampling kernels' footprint
    (libmoss_probe.so): loads per second at several occupancies, and the best."""
    import torch
    from paper_1509_08089_amd import probe
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    buf = torch.empty(max(1, footprint_bytes // 8), dtype=torch.int64, device="cuda")
    probe.moss_probe_fill(buf, 1)
    sweep = {}
    for w in waves_per_cu:
        blocks = cus * w // 4  # 256-lane blocks of four waves
        out = torch.empty(blocks * 256, dtype=torch.int64, device="cuda")
        steps = max(16, loads // (blocks * 256))
        probe.moss_probe_gather(buf, blocks, steps, out)  # warm-up (and brings the buffer into the caches)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            probe.moss_probe_gather(buf, blocks, steps, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        sweep[w] = blocks * 256 * steps / (ms / 1e3)
    best = max(sweep, key=sweep.get)
    return {"footprint_bytes": int(buf.numel() * 8), "probe_loads_per_s": sweep[best], "probe_waves_per_cu": best,
            "sweep_loads_per_s": {str(w): v for w, v in sweep.items()}}


def exact_counts(workload: str, sha: str, k: int):
    """Stored exact motif counts of the workload's graph (tests/golden), if any."""
    p = os.path.join(ROOT, "tests", "golden", f"exact_{workload.lower()}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("graph_sha256") != sha:
        return None
    return d.get("n4") if k == 4 else d.get("eta5")


def cpu_baseline(csr, cfg, seconds: float):
    import oracle
    cores = host_cores()
    t = time.time()
    og = oracle.Graph(csr)
    build_s = time.time() - t
    sid = oracle.MOSS4 if cfg["k"] == 4 else oracle.T5
    pair = (oracle.MOSS4, oracle.MOSS4MIN) if cfg.get("min") else (oracle.T5, oracle.PATH5)
    # calibrate, then run a bounded prefix of the sample stream
    n = 20_000 * cores
    t = time.time()
    og.run(sid, cfg["seed"], 0, n, cores)
    dt = max(time.time() - t, 1e-6)
    n = int(min(cfg["samples"], max(n, n * seconds / dt)))
    t = time.time()
    if cfg["k"] == 4 and not cfg.get("min"):
        og.run(oracle.MOSS4, cfg["seed"], 0, n, cores)
        done = n
    else:  # two samplers on half the samples each
        og.run(pair[0], cfg["seed"], 0, (n + 1) // 2, cores)
        og.run(pair[1], cfg["seed"], 0, n // 2, cores)
        done = n
    dt = time.time() - t
    return {"value": done / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"sample indices [0, {done}) of the same graph and seed ({done / cfg['samples']:.3%} of the "
                      f"workload), {cores} threads over contiguous index ranges; table build ({build_s:.2f} s) "
                      f"not included"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sampler shards by sample "
                                   "ranges with one histogram all-reduce, which is not built here",
                          "n_gpus": args.gpus}))
        return 2

    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.probe_only:
        print(json.dumps({"gather_probe": gather_ceiling(args.probe_only, waves_per_cu=(16,))}), flush=True)
        return 0

    import numpy as np
    import torch

    import graphgen as gg
    from paper_1509_08089_amd import moss

    torch.cuda.init()
    with_min = args.workload == "C2MIN"
    base = "C2" if with_min else args.workload  # graph, line counts and exact counts
    cfg = dict(gg.CONFIGS[base], min=with_min)
    log(f"[bench] generating {args.workload} graph")
    csr = cfg["graph"].build()
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
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"[bench] {args.steps} timed steps done")
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = K / (ms_per_step / 1e3)
    for r in results[1:]:
        assert np.array_equal(r.hits_np, results[0].hits_np)

    # roofline of the sampling kernel(s): algorithmic bytes per launch / average duration
    lc = json.load(open(os.path.join(ROOT, "tests", "golden", "line_counts.json")))[base]
    r0 = results[0]
    if with_min:
        alg_bytes = 64.0 * (r0.K[0] * lc["moss4"] + r0.K[1] * lc["moss4min"])
        kernel = "k_sample_moss4_moss4min"
    elif k == 4:
        alg_bytes = K * 64.0 * lc["moss4"]
        kernel = "k_sample_moss4"
    else:
        alg_bytes = 64.0 * (r0.K[0] * lc["t5"] + r0.K[1] * lc["path5"])
        kernel = "k_sample_t5_path5"
    kern_ms = sum(r.device_ms for r in results) / len(results)
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    traffic = measured_traffic(kernel, args.workload)
    traffic_gbs = traffic / (kern_ms / 1e3) / 1e9 if traffic else None
    line = {
        "metric": "graphlet samples/sec (4-,5-node) batched vs plain; serving p50/p99 latency",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT[args.workload]}", "k": k, "samples": K,
                   "n": csr.n, "m": csr.m, "graph_sha256": csr.sha256()[:16],
                   "step": "create over device CSR (validate) + build tables + sample/classify + finals"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": kernel, "kernel_ms": kern_ms,
                     "traffic_gbs": traffic_gbs, "traffic_frac": traffic_gbs / PEAK_HBM_GBS if traffic_gbs else None,
                     "alg_bytes_per_launch": alg_bytes,
                     "lines_per_sample": {kk: lc[kk] for kk in ("moss4", "moss4min", "t5", "path5") if kk in lc},
                     "kernel_samples_per_s": K / (kern_ms / 1e3)},
        "estimates": [float(x) for x in r0.estimate_np],
        "stderr_rel": [float(math.sqrt(v) / e) if e > 0 else None for v, e in zip(r0.variance_np, r0.estimate_np)],
    }
    exact = exact_counts(base, csr.sha256(), k)
    if exact is not None:
        line["exact"] = exact
        line["rel_error"] = [abs(e - x) / x if x else None for e, x in zip(line["estimates"], exact)]
    if not args.no_gather_probe:
        log("[bench] gather probe")
        h = moss.moss_graph_create_device(csr.n, csr.nnz, d_rp, d_col, 0, stream)
        try:
            moss.moss_build_tables(h, mask)
            fp = moss.moss_graph_get_info(h).sampling_bytes
        finally:
            moss.moss_graph_destroy(h)
        gc = gather_ceiling(fp)
        l1 = measured_l1_per_sample(kernel, args.workload)
        gc["kernel_l1_lines_per_sample"] = l1
        gc["kernel_l1_lines_per_s"] = l1 * K / (kern_ms / 1e3) if l1 else None
        gc["frac"] = gc["kernel_l1_lines_per_s"] / gc["probe_loads_per_s"] if l1 else None
        line["gather"] = gc
    if args.batched:
        line["batched"] = run_batched(moss, gg)
    if args.serve:
        line["serving"] = run_serving(moss, gg, args.serve_requests)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(csr, cfg, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


def run_batched(moss, gg):
    """256 requests over 32 graphs: one persistent launch vs one moss_estimate per request."""
    import numpy as np
    import torch
    specs, reqs = gg.batch_workload()
    log(f"[bench] batched: generating {len(specs)} graphs on the device")
    graphs = [moss.Graph.from_device(*s.build_device()) for s in specs]
    torch.cuda.synchronize()
    q = [(graphs[r.graph].h, r.k, r.samples, r.seed, 0) for r in reqs]
    total = sum(r.samples for r in reqs)
    for g in graphs:
        g.build_tables()
    def timed(fn, reps=3):  # median wall time of `reps` calls after one warm-up call
        out = fn()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            ts.append(time.perf_counter() - t)
        return sorted(ts)[len(ts) // 2], out

    t_batch, got = timed(lambda: moss.moss_estimate_batch(q))
    t_plain, alone = timed(lambda: [moss.moss_estimate(*x) for x in q])
    same = all(np.array_equal(a.hits_np, b.hits_np) for a, b in zip(alone, got))
    best, ms = moss.moss_autotune(q)
    t_tuned, got2 = timed(lambda: moss.moss_estimate_batch(q))
    same = same and all(np.array_equal(a.hits_np, b.hits_np) for a, b in zip(alone, got2))
    moss.moss_set_tuning(0, 0, 0)
    return {"requests": len(q), "graphs": len(graphs), "samples": total,
            "batched_samples_per_s": total / t_batch, "plain_samples_per_s": total / t_plain,
            "tuned_samples_per_s": total / t_tuned, "speedup": t_plain / t_batch,
            "tuning": {"tile_samples": best.tile_samples, "blocks_per_cu": best.blocks_per_cu},
            "identical_results": bool(same)}


def run_serving(moss, gg, n_requests):
    import torch
    specs, reqs = gg.serving_workload(n_requests=n_requests)
    log(f"[bench] serving: generating {len(specs)} graphs on the device")
    graphs = [moss.Graph.from_device(*s.build_device()) for s in specs]
    torch.cuda.synchronize()
    srv = moss.moss_server_create(0, 256, 1 << 22)
    try:
        ids = [moss.moss_server_add_graph(srv, g.h) for g in graphs]
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            now = time.perf_counter() - t0
            if r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            tickets.append(moss.moss_server_submit(srv, ids[r.graph], r.k, r.samples, r.seed))
        for tk in tickets:
            moss.moss_server_wait(srv, tk, -1)
        wall = time.perf_counter() - t0
        st = moss.moss_server_stats_get(srv)
    finally:
        moss.moss_server_destroy(srv)
    offered = sum(r.samples for r in reqs) / reqs[-1].arrival_s
    return {"requests": len(reqs), "graphs": len(graphs), "rate_req_s": len(reqs) / reqs[-1].arrival_s,
            "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "samples_per_s": st.samples_per_s,
            "offered_samples_per_s": offered, "wall_s": wall, "iterations": st.iterations}


if __name__ == "__main__":
    sys.exit(main())
