#!/usr/bin/env python3
"""Write the expected survey results of the full-size workloads.

Runs only the CPU oracle on the seeded synthetic inputs and stores its
counters as JSON next to this script (golden_w<k>_s<scale>.json).  The GPU
tests regenerate the same inputs and compare against these files.

    python tests/golden/make_golden.py 2        # workload 2 at its scale
    python tests/golden/make_golden.py 3 --scale 26
    python tests/golden/make_golden.py 2 --extended   # golden_ext_w2_s22.json

--extended stores the extended outputs instead: Algorithm 3's max-edge bins,
the degree-log table and the directed census (the raw edges read as arcs
src -> dst), and checksums of the per-vertex and per-edge participation
counts (see participation_checksums).
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


def golden_path(workload: int, scale: int, extended: bool = False) -> str:
    return os.path.join(HERE, "golden_%sw%d_s%d.json" % ("ext_" if extended else "", workload, scale))


def max_edge_shift(w) -> int:
    """Bins of 2^shift that span the workload's time range with 1024 bins."""
    bits = w.graph.ts[1] if w.graph.ts[0] == "uniform" else 31
    return max(0, bits - 10)


def participation_checksums(n, vcount, lo, hi, ecount) -> dict:
    """Order-free digests of participation counts: their sums, sums of
    squares, and sums weighted by the vertex id or by the edge's endpoint
    ids, all modulo 2^64."""
    vc = np.asarray(vcount, np.uint64)
    ec = np.asarray(ecount, np.uint64)
    ids = np.arange(len(vc), dtype=np.uint64)
    key = np.asarray(lo, np.uint64) * np.uint64(n) + np.asarray(hi, np.uint64)
    with np.errstate(over="ignore"):
        return {"vertex_sum": int(vc.sum(dtype=np.uint64)), "vertex_sq": int((vc * vc).sum(dtype=np.uint64)),
                "vertex_weighted": int((vc * (ids * np.uint64(2654435761) + np.uint64(1))).sum(dtype=np.uint64)),
                "edge_sum": int(ec.sum(dtype=np.uint64)), "edge_sq": int((ec * ec).sum(dtype=np.uint64)),
                "edge_weighted": int((ec * (key * np.uint64(2654435761) + np.uint64(1))).sum(dtype=np.uint64)),
                "edges_with_triangles": int((ec > 0).sum())}


def extended(w, threads):
    g = w.graph
    data = synth.generate(g)
    u, v, t, d = oracle.clean(g.n, data["src"], data["dst"], data["ts"], directions=True)
    shift = max_edge_shift(w)
    t0 = time.time()
    r = oracle.survey_clean(g.n, u, v, t, data["vlab"], outputs=("count", "max_edge", "degree_table", "directed"),
                            n_labels=w.n_labels, max_edge_shift=shift, edir=d, threads=threads)
    t1 = time.time()
    vc, (pu, pv, pt, ec) = oracle.participation(g.n, data["src"], data["dst"], data["ts"], data["vlab"],
                                                n_labels=w.n_labels, threads=threads)
    t2 = time.time()
    deg = np.asarray(r["degree_table"])
    return {
        "about": "Oracle extended outputs of the seeded synthetic workload %d (%s); written by "
                 "tests/golden/make_golden.py --extended, which calls only the oracle and the input generator."
                 % (w.number, w.name),
        "workload": w.number, "name": w.name, "scale": g.scale, "seed": g.seed, "n_labels": w.n_labels,
        "m": int(len(u)), "triangles": r["triangles"], "max_edge_shift": shift,
        "max_edge": [int(x) for x in r["max_edge"]],
        "degree_table": {str(i): int(deg[i]) for i in np.nonzero(deg)[0]},
        "directed": [int(x) for x in r["directed"]],
        "participation": participation_checksums(g.n, vc, pu, pv, ec),
        "oracle_seconds": {"survey": round(t1 - t0, 2), "participation": round(t2 - t1, 2)},
        "host_threads": threads or os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", type=int)
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--extended", action="store_true")
    a = ap.parse_args()
    w = synth.workload(a.workload, scale=a.scale)
    if a.extended:
        out = extended(w, a.threads)
        path = golden_path(w.number, w.graph.scale, extended=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print("wrote", path, out["triangles"], out["oracle_seconds"])
        return
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
