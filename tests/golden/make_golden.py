"""Writes the stored reference values under tests/golden/ using only the oracle and
the seeded input generators.

  line_counts.json  mean number of distinct 64-byte lines one sample reads (binary
                    searches as in Section 4.1.3, no reuse between samples), per
                    workload and sampler, over the first `samples` indices of seed 1;
                    64 B times this is the roofline's algorithmic bytes per sample
  exact_c1.json     exact 4- and 5-node CIS counts of the C1 graph (enumeration)
  exact_c2.json     exact 4-node counts of the C2 graph (non-induced patterns converted
                    through the containment matrix; enumeration is infeasible there)

Usage: python tests/golden/make_golden.py [--skip-exact5] [--only lines|c1|c2] [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

SAMPLERS = {"moss4": oracle.MOSS4, "moss4min": oracle.MOSS4MIN, "t5": oracle.T5, "path5": oracle.PATH5}


def line_counts(samples: int) -> dict:
    out = {}
    for name in ("C1", "C2", "C3"):
        cfg = gg.CONFIGS[name]
        g = cfg["graph"].build()
        og = oracle.Graph(g)
        entry = {"graph_sha256": g.sha256(), "n": g.n, "m": g.m, "seed": cfg["seed"], "samples": samples}
        for sname, sid in SAMPLERS.items():
            if (cfg["k"] == 4) != (sname in ("moss4", "moss4min")):
                continue
            entry[sname] = og.line_count(sid, cfg["seed"], 0, samples)
        out[name] = entry
        print(name, entry, flush=True)
    return out


def exact_c1(with5: bool, threads: int) -> dict:
    g = gg.config_graph("C1")
    og = oracle.Graph(g)
    t = time.time()
    c4 = [int(x) for x in og.count_cis(4, threads)[1:7]]
    res = {"graph_sha256": g.sha256(), "n4": c4, "seconds4": round(time.time() - t, 1), "threads": threads}
    if with5:
        t = time.time()
        res["eta5"] = [int(x) for x in og.count_cis(5, threads)[1:22]]
        res["seconds5"] = round(time.time() - t, 1)
    res.update(og.totals())
    return res


def exact_c2() -> dict:
    g = gg.config_graph("C2")
    og = oracle.Graph(g)
    t = time.time()
    n4 = [int(x) for x in og.count4_exact()[1:7]]
    return {"graph_sha256": g.sha256(), "n4": n4, "seconds": round(time.time() - t, 1)}


def write(name: str, obj: dict):
    """Writes tests/golden/<name> only once its values are computed (atomically)."""
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
    os.replace(path + ".tmp", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=200_000)
    ap.add_argument("--skip-exact5", action="store_true")
    ap.add_argument("--only", choices=["lines", "c1", "c2"], default=None)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1, help="threads of the enumeration")
    a = ap.parse_args()
    if a.only in (None, "lines"):
        write("line_counts.json", line_counts(a.samples))
    if a.only in (None, "c1"):
        write("exact_c1.json", exact_c1(not a.skip_exact5, a.threads))
    if a.only in (None, "c2"):
        write("exact_c2.json", exact_c2())


if __name__ == "__main__":
    main()
