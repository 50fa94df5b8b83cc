#!/usr/bin/env python3
"""Write the expected survey results of the full-size workloads.

Runs only the CPU oracle on the seeded synthetic inputs and stores its
counters as JSON next to this script (golden_w<k>_s<scale>.json).  The GPU
tests regenerate the same inputs and compare against these files.

    python tests/golden/make_golden.py 2        # workload 2 at its scale
    python tests/golden/make_golden.py 3 --scale 26
"""
import argparse
import gc
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

ALL_OUT = ("count", "close_hist", "label_table", "spread_count", "open_close")


def golden_path(workload: int, scale: int) -> str:
    return os.path.join(HERE, "golden_w%d_s%d.json" % (workload, scale))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", type=int)
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    w = synth.workload(a.workload, scale=a.scale)
    g = w.graph
    t0 = time.time()
    data = synth.generate(g)
    t1 = time.time()
    u, v, t = oracle.clean(g.n, data["src"], data["dst"], data["ts"])
    vlab = data["vlab"]
    del data
    gc.collect()
    t2 = time.time()
    spread = w.spread_lt or (1 << 16)
    r = oracle.survey_clean(g.n, u, v, t, vlab, outputs=ALL_OUT, n_labels=w.n_labels, spread_lt=spread,
                            threads=a.threads)
    t3 = time.time()
    out = {
        "about": "Oracle survey of the seeded synthetic workload %d (%s); written by tests/golden/make_golden.py, "
                 "which calls only the oracle and the input generator." % (w.number, w.name),
        "workload": w.number, "name": w.name, "kind": g.kind, "scale": g.scale, "edge_factor": g.edge_factor,
        "seed": g.seed, "ts": list(g.ts), "labels": list(g.labels), "n_labels": w.n_labels, "spread_lt": spread,
        "m": int(len(u)), "triangles": r["triangles"], "wedges_degree_id_order": r["wedges"],
        "spread_count": r["spread_count"], "close_hist": [int(x) for x in r["close_hist"]],
        "label_table": [int(x) for x in r["label_table"]],
        "open_close": [int(x) for x in np.asarray(r["open_close"]).ravel()],
        "oracle_seconds": {"generate": round(t1 - t0, 2), "clean": round(t2 - t1, 2), "survey": round(t3 - t2, 2)},
        "host_threads": a.threads or os.cpu_count(),
    }
    with open(golden_path(w.number, g.scale), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", golden_path(w.number, g.scale), out["triangles"], out["oracle_seconds"])


if __name__ == "__main__":
    main()
