"""The benchmark's counter arithmetic on synthetic rocprofv3 output (no GPU): the per-launch
sums of the sampling launch's kernels, the request-size weighting of the bytes past the
L2s, the L2 clock, busy fraction and hit rate, and the roofline's choice between the
fabric and the L2-request ceilings."""
import csv
import os
import re

import pytest

import bench


def _write_run(d, launches, counters, trace):
    """One rocprofv3 pass: counters = {(kernel, counter): value per dispatch}, each kernel
    dispatched once per launch; trace = {kernel: duration_ns}."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        disp = 0
        for _ in range(launches):
            for kn in sorted({k for k, _ in counters}):
                disp += 1
                for (k, cn), v in counters.items():
                    if k == kn:
                        w.writerow({"Dispatch_Id": disp, "Kernel_Name": kn, "Counter_Name": cn, "Counter_Value": v})
    with open(os.path.join(d, "x_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 1_000_000
        for _ in range(launches):
            for kn, ns in trace.items():
                w.writerow({"Kernel_Name": kn, "Start_Timestamp": t, "End_Timestamp": t + ns})
                t += ns + 500


def _values(summary):
    out = {}
    for line in summary.splitlines():
        m = re.match(r"^([a-z0-9_]+(?: [A-Za-z0-9_]+)?):\s*([0-9a-fA-F.eE+-]+)\s*$", line.strip())
        if m:
            out[m.group(1)] = m.group(2)
    return out


BATCH = "moss::k_batch(moss::SamplerView const*, moss::BatchItem const*, unsigned int*, unsigned long long*)"
SORTED = "void moss::k_sample_sorted<4>(moss::SamplerView, unsigned long)"
OTHER = "moss::k_edge_insert(long, int const*)"  # not a kernel of the sampling launch


def _runs(tmp_path, launches=2, reads128=650):
    a = {(BATCH, "TCC_EA0_RDREQ_sum"): 350 + reads128, (BATCH, "TCC_EA0_RDREQ_32B_sum"): 100,
         (BATCH, "TCC_EA0_RDREQ_64B_sum"): 200, (BATCH, "TCC_EA0_RDREQ_128B_sum"): reads128,
         (SORTED, "TCC_EA0_RDREQ_sum"): 400, (SORTED, "TCC_EA0_RDREQ_128B_sum"): 400,
         (OTHER, "TCC_EA0_RDREQ_sum"): 10 ** 9, (OTHER, "TCC_EA0_RDREQ_128B_sum"): 10 ** 9}
    b = {(BATCH, "TCC_REQ_sum"): 5000, (BATCH, "TCC_CYCLE_sum"): 128 * 2.0e6, (BATCH, "TCC_BUSY_sum"): 64 * 2.0e6,
         (SORTED, "TCC_REQ_sum"): 3000, (OTHER, "TCC_REQ_sum"): 10 ** 9}
    c = {(BATCH, "TCC_EA0_WRREQ_sum"): 30, (BATCH, "TCC_EA0_WRREQ_64B_sum"): 10,
         (BATCH, "TCC_HIT_sum"): 750, (BATCH, "TCC_MISS_sum"): 250}
    trace = {BATCH: 800_000, SORTED: 200_000, OTHER: 5_000_000}  # ns per launch
    dirs = []
    for name, counters in (("A", a), ("B", b), ("C", c)):
        d = str(tmp_path / name)
        _write_run(d, launches, counters, trace)
        dirs.append(d)
    return dirs


def test_summary_per_launch_and_weighted_bytes(tmp_path):
    dirs = _runs(tmp_path, launches=2)
    v = _values(bench.summarize_counters(dirs, "TEST", 2, source_sha="feedface"))
    assert v["kernel_source_sha"] == "feedface"
    # the launch's kernels only (k_edge_insert left out), per launch
    assert float(v["launch_kernel_us"]) == pytest.approx(1000.0)  # 800 + 200 us, three traced runs
    assert float(v["per_launch TCC_EA0_RDREQ_sum"]) == pytest.approx(1400)
    assert float(v["tcc_req_per_launch"]) == pytest.approx(8000)
    # reads weighted by request size, writes 32 B unless counted as 64 B
    assert float(v["read_bytes_per_launch"]) == pytest.approx(32 * 100 + 64 * 200 + 128 * (650 + 400))
    assert float(v["rdreq_unsized_per_launch"]) == pytest.approx(1400 - 100 - 200 - 1050)
    assert float(v["write_bytes_per_launch"]) == pytest.approx(32 * 20 + 64 * 10)
    assert float(v["fabric_bytes_per_launch"]) == pytest.approx(32 * 100 + 64 * 200 + 128 * 1050 + 32 * 20 + 64 * 10)
    # 128 channels x 2e6 cycles in 1000 us of kernel time: 2 GHz; half the cycles busy
    assert float(v["l2_clock_hz"]) == pytest.approx(2.0e9)
    assert float(v["l2_busy_frac"]) == pytest.approx(0.5)
    assert float(v["l2_hit_rate"]) == pytest.approx(0.75)


@pytest.mark.parametrize("reads128,bound", [(650, "l2"), (10 ** 7, "hbm")])
def test_roofline_takes_the_binding_ceiling(tmp_path, monkeypatch, reads128, bound):
    """Both fractions scale with 1 / launch time; which binds depends on the counters:
    8,000 L2 requests against a few hundred KB past the L2s is L2-bound, ten million
    128-byte reads fabric-bound."""
    device_ms = 1.0
    dirs = _runs(tmp_path, launches=1, reads128=reads128)
    summary = bench.summarize_counters(dirs, "TEST", 1, source_sha="feedface")
    root = tmp_path / "root"
    (root / "profiles").mkdir(parents=True)
    (root / "profiles" / "counters_TEST.md").write_text(summary)
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "feedface")
    r = bench.roofline("TEST", device_ms, None, 1000.0)
    secs = device_ms / 1e3
    fabric = 32 * 100 + 64 * 200 + 128 * (reads128 + 400) + 32 * 20 + 64 * 10
    fab_frac = fabric / secs / 1e9 / bench.PEAK_HBM_GBS
    l2_frac = 8000 / secs / (bench.L2_CHANNELS * 2.0e9)
    assert r["fabric"]["frac"] == pytest.approx(fab_frac)
    assert r["l2"]["frac"] == pytest.approx(l2_frac)
    assert r["frac"] == pytest.approx(max(fab_frac, l2_frac))
    assert r["bound"] == ("hbm" if fab_frac >= l2_frac else "l2") == bound
    assert r["traffic"] == pytest.approx(fabric)
    assert r["l2"]["requests_per_sample"] == pytest.approx(8.0)


def test_roofline_without_a_current_summary(tmp_path, monkeypatch):
    """A summary taken on other kernel sources is not used: frac and traffic are null."""
    dirs = _runs(tmp_path, launches=1)
    root = tmp_path / "root"
    (root / "profiles").mkdir(parents=True)
    (root / "profiles" / "counters_TEST.md").write_text(
        bench.summarize_counters(dirs, "TEST", 1, source_sha="0000000000000000"))
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "feedface")
    r = bench.roofline("TEST", 1.0, None, 1000.0)
    assert r["frac"] is None and r["traffic"] is None
