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
src -> dst), and digests of the per-vertex and per-edge participation
counts (see participation_checksums; their SHA-256 digests compare every
count).

    python tests/golden/make_golden.py 2 --max-edge-exact   # golden_maxe_w2_s22.json
    python tests/golden/make_golden.py 4 --batch      # golden_batch_w4.json
    python tests/golden/make_golden.py 5 --served     # golden_served_pool.json

--max-edge-exact stores Algorithm 3's exact counting set (every distinct
largest edge time over the distinct-label triangles, with its count): its
size, its total, SHA-256 digests of the ascending values (uint32 little
endian) and of their counts (uint64 little endian), and every 10000th entry.

--batch surveys every graph of the 20,000-graph batch on its own (one oracle
process per graph, in a pool) and stores every graph's triangle count, the
sum of all closure histograms, and the full histogram of every 50th graph
and of every scale-16 member.  --served stores, for each graph of the served
pool (R-MAT scales 16..20), the oracle's answers to seeded requests of the
served kinds: a full survey, a time window and a label predicate.
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
    """Digests of participation counts: their sums, sums of squares, and
    sums weighted by the vertex id or by the edge's endpoint ids, all modulo
    2^64; and SHA-256 of every count in a canonical order (vertices by id,
    edges by (lower id, higher id), little-endian uint64), which compares
    the counts element by element."""
    import hashlib
    vc = np.asarray(vcount, np.uint64)
    ec = np.asarray(ecount, np.uint64)
    ids = np.arange(len(vc), dtype=np.uint64)
    key = np.asarray(lo, np.uint64) * np.uint64(n) + np.asarray(hi, np.uint64)
    order = np.argsort(key, kind="stable")
    with np.errstate(over="ignore"):
        return {"vertex_sum": int(vc.sum(dtype=np.uint64)), "vertex_sq": int((vc * vc).sum(dtype=np.uint64)),
                "vertex_weighted": int((vc * (ids * np.uint64(2654435761) + np.uint64(1))).sum(dtype=np.uint64)),
                "edge_sum": int(ec.sum(dtype=np.uint64)), "edge_sq": int((ec * ec).sum(dtype=np.uint64)),
                "edge_weighted": int((ec * (key * np.uint64(2654435761) + np.uint64(1))).sum(dtype=np.uint64)),
                "edges_with_triangles": int((ec > 0).sum()),
                "vertex_sha256": hashlib.sha256(vc.astype("<u8").tobytes()).hexdigest(),
                "edge_sha256_by_pair": hashlib.sha256(ec[order].astype("<u8").tobytes()).hexdigest()}


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


def max_edge_exact(w, threads):
    import hashlib
    g = w.graph
    data = synth.generate(g)
    t0 = time.time()
    vals, cnts = oracle.max_edge_counts(g.n, data["src"], data["dst"], data["ts"], data["vlab"],
                                        n_labels=w.n_labels, threads=threads)
    t1 = time.time()
    pick = np.arange(0, len(vals), 10000)
    return {
        "about": "Oracle exact counting set of Algorithm 3 for the seeded synthetic workload %d (%s); written by "
                 "tests/golden/make_golden.py --max-edge-exact, which calls only the oracle and the input generator."
                 % (w.number, w.name),
        "workload": w.number, "name": w.name, "scale": g.scale, "seed": g.seed, "n_labels": w.n_labels,
        "n_values": int(len(vals)), "total": int(cnts.sum(dtype=np.uint64)),
        "sha256_values": hashlib.sha256(vals.astype("<u4").tobytes()).hexdigest(),
        "sha256_counts": hashlib.sha256(cnts.astype("<u8").tobytes()).hexdigest(),
        "sample_stride": 10000,
        "sample": [[int(i), int(vals[i]), int(cnts[i])] for i in pick],
        "oracle_seconds": round(t1 - t0, 2), "host_threads": threads or os.cpu_count(),
    }


BATCH_STRIDE = 50


def batch_sample(specs) -> list:
    """Graphs whose full histograms are stored: every BATCH_STRIDE-th graph
    and every member of the largest scale."""
    top = max(s.scale for s in specs)
    return sorted({g for g in range(0, len(specs), BATCH_STRIDE)} |
                  {g for g, s in enumerate(specs) if s.scale == top})


def _batch_member(arg):
    g, spec = arg
    d = synth.generate(spec)
    r = oracle.survey(spec.n, d["src"], d["dst"], d["ts"], d["vlab"], outputs=("count", "close_hist"),
                      n_labels=int(spec.labels[1]), threads=1)
    return g, int(r["triangles"]), [int(x) for x in r["close_hist"]], int(r["m"])


def batch(w, procs):
    """Oracle survey of every graph of the batched workload, each alone."""
    import multiprocessing as mp
    ex = w.extra
    specs = synth.batch_specs(ex["n_graphs"], scale_lo=ex["scale_lo"], scale_hi=ex["scale_hi"],
                              ef_lo=ex["ef_lo"], ef_hi=ex["ef_hi"])
    order = sorted(range(len(specs)), key=lambda g: -specs[g].n_edges)
    tri = [0] * len(specs)
    edges = [0] * len(specs)
    hist = {}
    total = np.zeros(32, np.uint64)
    t0 = time.time()
    # one thread per worker process: the generator's and the oracle's
    # OpenMP runtimes read this when they start in the (spawned) workers
    os.environ["OMP_NUM_THREADS"] = "1"
    with mp.get_context("spawn").Pool(procs or os.cpu_count()) as pool:
        for k, (g, t, h, m) in enumerate(pool.imap_unordered(_batch_member, [(g, specs[g]) for g in order],
                                                             chunksize=4)):
            tri[g], edges[g] = t, m
            hist[g] = h
            total += np.array(h, np.uint64)
            if k % 1000 == 0:
                print("  %d graphs surveyed (%.0f s)" % (k, time.time() - t0), flush=True)
    sample = batch_sample(specs)
    return {
        "about": "Oracle survey of every graph of the seeded batched workload %d (%s), each graph alone; written "
                 "by tests/golden/make_golden.py --batch, which calls only the oracle and the input generator."
                 % (w.number, w.name),
        "workload": w.number, "name": w.name, "n_graphs": len(specs), "outputs": ["count", "close_hist"],
        "n_labels": w.n_labels, "scale_range": [ex["scale_lo"], ex["scale_hi"]],
        "edge_factor_range": [ex["ef_lo"], ex["ef_hi"]],
        "raw_edges": int(sum(s.n_edges for s in specs)), "edges": int(sum(edges)),
        "triangles_total": int(sum(tri)), "triangles": tri,
        "close_hist_total": [int(x) for x in total],
        "close_hist_sample": {str(g): hist[g] for g in sample},
        "oracle_seconds": round(time.time() - t0, 1), "host_processes": procs or os.cpu_count(),
    }


def served_pool_specs(w):
    """The served pool graphs (R-MAT scales lo..hi, times uniform on
    [0, 2^31), labels uniform on 0..L-1) as the benchmark builds them."""
    ex = w.extra
    return [synth.GraphSpec("rmat", sc, 16, synth.MASTER_SEED + 50 + k, ("uniform", 31), ("uniform", w.n_labels))
            for k, sc in enumerate(range(ex["pool_scale_lo"], ex["pool_scale_hi"] + 1))]


def served_requests(L, seed):
    """Seeded requests of the served kinds on one graph: a full survey
    (closure histogram, label table, spread count), a closed time window of
    log-uniform width in [2^12, 2^31], and a label predicate (each multiset
    bit set with probability 1/2)."""
    rng = np.random.default_rng(seed)
    n_tab = (L + 2) * (L + 1) * L // 6
    width = int(2 ** (12 + 19 * rng.random()))
    lo = int(rng.integers(0, 1 << 31))
    mask = [int(i) for i in np.nonzero(rng.random(n_tab) < 0.5)[0]]
    return [dict(outputs=["count", "close_hist", "label_table", "spread_count"],
                 spread_lt=int(1 << int(rng.integers(16, 28)))),
            dict(outputs=["count", "close_hist"], window=[lo, min(lo + width, (1 << 32) - 1)]),
            dict(outputs=["count"], label_mask=mask)]


def served(w, threads):
    out = []
    for k, spec in enumerate(served_pool_specs(w)):
        d = synth.generate(spec)
        u, v, t = oracle.clean(spec.n, d["src"], d["dst"], d["ts"])
        reqs = []
        for rq in served_requests(w.n_labels, synth.MASTER_SEED + 500 + k):
            kw = dict(rq)
            kw["outputs"] = tuple(kw["outputs"])
            r = oracle.survey_clean(spec.n, u, v, t, d["vlab"], n_labels=w.n_labels, threads=threads, **kw)
            res = {"triangles": int(r["triangles"])}
            if "close_hist" in rq["outputs"]:
                res["close_hist"] = [int(x) for x in r["close_hist"]]
            if "label_table" in rq["outputs"]:
                res["label_table"] = [int(x) for x in r["label_table"]]
            if "spread_count" in rq["outputs"]:
                res["spread_count"] = int(r["spread_count"])
            reqs.append({"request": rq, "result": res})
        print("  pool graph %d (scale %d): %d triangles" % (k, spec.scale, reqs[0]["result"]["triangles"]),
              flush=True)
        out.append({"scale": spec.scale, "edge_factor": spec.edge_factor, "seed": spec.seed, "ts": list(spec.ts),
                    "labels": list(spec.labels), "m": int(len(u)), "requests": reqs})
    return {
        "about": "Oracle answers to seeded served requests on the pool graphs of workload %d (%s); written by "
                 "tests/golden/make_golden.py --served, which calls only the oracle and the input generator."
                 % (w.number, w.name),
        "workload": w.number, "n_labels": w.n_labels, "graphs": out,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", type=int)
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--extended", action="store_true")
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--served", action="store_true")
    ap.add_argument("--max-edge-exact", action="store_true")
    a = ap.parse_args()
    w = synth.workload(a.workload, scale=a.scale)
    if a.max_edge_exact:
        out = max_edge_exact(w, a.threads)
        path = os.path.join(HERE, "golden_maxe_w%d_s%d.json" % (w.number, w.graph.scale))
        with open(path, "w") as f:
            json.dump(out, f, separators=(",", ":"))
        print("wrote", path, out["n_values"], out["total"], out["oracle_seconds"])
        return
    if a.batch or a.served:
        out = batch(w, a.threads) if a.batch else served(w, a.threads)
        path = os.path.join(HERE, "golden_batch_w4.json" if a.batch else "golden_served_pool.json")
        with open(path, "w") as f:
            json.dump(out, f, separators=(",", ":") if a.batch else (", ", ": "), indent=None if a.batch else 1)
        print("wrote", path)
        return
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
