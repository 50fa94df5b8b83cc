#!/usr/bin/env python3
"""Benchmark of the metadata triangle survey on one MI355X.

One step is one pass of the whole hot path over the resident raw edge list:
build the degree-ordered directed graph (canonicalise, sort, dedup with the
earliest time, degree order, orient, CSR with co-located metadata, in-edge
index, tile plan), survey it (intersection kernels with the fused reducer)
and read the counters back.  The raw edges are generated once (seeded
synthetic R-MAT input) and are resident in HBM before the timed region.

Prints one JSON line.  `value` is triangles surveyed per second of whole
steps.  The `roofline` object covers the dominant survey kernel: its
algorithmic bytes per launch divided by its average launch time, measured
with HIP events recorded on the stream the kernel is launched on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "triangles surveyed/s + HBM GB/s at R-MAT scale 26; p50/p99 survey latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2107_12330_amd", "csrc", "survey.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "survey_traffic.json")
CLASS_NAMES = ("tiny (d+(q) <= 51)", "small (d+(q) <= 819)", "large (d+(q) <= 3276)",
               "huge (d+(q) > 3276, in pieces of Adj+(q))")
VARIANT_NAMES = {1: "LDS cuckoo tables, one per wave", 2: "LDS cuckoo tables, one per workgroup",
                 3: "HBM binary search, a workgroup per tile", 4: "HBM binary search, a wave per tile"}


def resolve_variant(c: int, v: int) -> int:
    """The variant a class runs with (the library's default when 0)."""
    return v if v else {0: 1, 1: 2, 2: 2, 3: 2}[c]


def kernel_key(c: int, v: int, meta: bool, form: int = 0) -> str:
    """Template arguments of the survey kernel that serves class c under
    variant v, as in the rocprofv3 kernel name (spaces removed).  form: 0 the
    plain survey, 1 the extended reductions, 2 participation; the next
    argument marks the huge class's kernels, which walk pieces of Adj+(q);
    the last one the doubled hit ring, which the 1024-thread workgroups of
    the plain metadata survey take wherever their counters leave the LDS for
    it (every output set of these workloads)."""
    v = resolve_variant(c, v)
    log_slots, block, wave = {1: (6, 256, "true"), 2: (12, 1024, "false") if c >= 2 else (10, 256, "false"),
                              3: (0, 256, "false"), 4: (0, 256, "true")}[v]
    wide = meta and form == 0 and wave == "false" and block == 1024
    return "survey_kernel<%d,%d,%s,%s,false,false,%d,%s,%s>" % (
        log_slots, block, wave, "true" if meta else "false", form, "true" if c == 3 else "false",
        "true" if wide else "false")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("survey.hip", "graph.hpp", "plan.hpp", "multi.hpp", "tp_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2107_12330_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(st: dict, c: int, meta: bool, hits: int) -> int:
    """Bytes the survey of target class c must move, per launch, by the
    work model of the q-centric survey: per wedge check the candidate r
    (4 B); per hit the time of edge (p, r) (4 B, metadata surveys only); per
    staged out-list entry of a target its rank, and for metadata surveys its
    edge time and label (4 or 9 B); per in-edge record 8 B; per tile its two
    row pointers (16 B)."""
    per_staged = 9 if meta else 4
    return (4 * st["class_probes"][c] + (4 * hits if meta else 0) + per_staged * st["class_staged"][c]
            + 8 * st["class_records"][c] + 16 * st["class_tiles"][c])


def batch_work(st: dict, triangles: int, survey_ms: float, meta: bool) -> dict:
    """Work of a batch survey per target class, and the whole survey's bytes
    by the work model (all triangles are hits of some class) against its
    recorded time and the 8 TB/s peak."""
    b_alg = sum(algorithmic_bytes(st, c, meta, 0) for c in range(4)) + (4 * triangles if meta else 0)
    return {"class_probes": st["class_probes"], "class_records": st["class_records"],
            "class_staged": st["class_staged"], "survey_algorithmic_bytes": b_alg,
            "survey_frac": round(b_alg / (survey_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}


def loaded_bytes(st: dict, c: int, meta: bool) -> int:
    """Bytes the kernel of class c loads by design: every candidate's rank
    and, for metadata surveys, its edge time (a hit rate near one in five
    touches nearly every line of times anyway), each staged entry, the
    in-edge records with their time(p, q) gather, and the tiles."""
    per_probe = 8 if meta else 4
    per_staged = 9 if meta else 4
    return (per_probe * st["class_probes"][c] + per_staged * st["class_staged"][c] + 16 * st["class_records"][c]
            + 32 * st["class_tiles"][c])


def load_traffic(key: str, workload_name: str):
    """HBM bytes per launch of the kernel `key` from the committed rocprofv3
    counter summary, if it was taken on the current kernel source and this
    workload (else None)."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_source_hash() or rec.get("workload") != workload_name:
        return None
    v = rec.get("kernels", {}).get(key)
    return None if v is None else int(v["hbm_bytes_per_launch"])


# The oracle's own run of the full scale-26 workload (single-threaded clean,
# then the survey on 8 threads), as stored beside its result by
# tests/golden/make_golden.py on the 8-core build host.
FULL_C3_ORACLE = {"triangles": 49164311615, "clean_s": 297.47, "survey_s": 1968.17, "threads": 8,
                  "host": "8-core Intel Xeon Processor @ 2.70GHz"}


def cpu_baseline(scale: int, threads: int) -> dict:
    """The oracle (clean + survey) on a bounded sample: the same recipe at a
    smaller R-MAT scale, timed on this host's cores."""
    import oracle
    import synth
    w = synth.workload(3, scale=scale)
    g = synth.generate(w.graph)
    t0 = time.perf_counter()
    u, v, t = oracle.clean(g["n"], g["src"], g["dst"], g["ts"])
    r = oracle.survey_clean(g["n"], u, v, t, g["vlab"], outputs=w.outputs, n_labels=4, spread_lt=w.spread_lt,
                            threads=threads)
    dt = time.perf_counter() - t0
    full = FULL_C3_ORACLE
    return {"value": r["triangles"] / dt, "unit": "triangles/s", "cores": threads, "kind": "oracle",
            "sample": "R-MAT scale %d of the scale-26 recipe (%s: bursty times, labels 0..3, same outputs), not "
                      "the scale-26 input itself: full oracle pipeline (single-threaded clean, then orient + "
                      "survey on %d threads), %d triangles in %.2f s"
                      % (scale, w.name, threads, r["triangles"], dt),
            "full_config_oracle": dict(full, triangles_per_s=round(full["triangles"] /
                                                                   (full["clean_s"] + full["survey_s"]), 1),
                                       input="rmat-s26-bursty (the bench workload itself)")}


def oracle_table(threads: int, workloads=(1, 2), sample_scale: int | None = None) -> dict:
    """The oracle's own times per workload, on this host: the clean
    (single-threaded) and the survey (orient + intersect + reduce) timed
    apart, the survey on one thread and on `threads`.  Workloads 1 and 2 at
    their full sizes; optionally the scale-26 recipe at `sample_scale` (the
    oracle does not finish the full size in a few minutes)."""
    import oracle
    import synth
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    rows = []
    cases = [(wl, None) for wl in workloads] + ([(3, sample_scale)] if sample_scale else [])
    for wl, scale in cases:
        w = synth.workload(wl, scale=scale)
        g = synth.generate(w.graph)
        L = int(w.graph.labels[1])
        t0 = time.perf_counter()
        u, v, t = oracle.clean(g["n"], g["src"], g["dst"], g["ts"])
        clean_s = time.perf_counter() - t0
        row = {"workload": wl, "scale": w.graph.scale, "raw_edges": int(len(g["src"])), "edges": int(len(u)),
               "outputs": list(w.outputs), "clean_s": round(clean_s, 3)}
        for th in sorted({1, threads}):
            t0 = time.perf_counter()
            r = oracle.survey_clean(g["n"], u, v, t, g["vlab"], outputs=w.outputs, n_labels=L,
                                    spread_lt=w.spread_lt, threads=th)
            dt = time.perf_counter() - t0
            row["survey_s_%d_threads" % th] = round(dt, 3)
            row["triangles"] = int(r["triangles"])
            log("oracle workload %d scale %d: clean %.2f s, survey on %d threads %.2f s"
                % (wl, w.graph.scale, clean_s, th, dt))
        rows.append(row)
        del g, u, v, t
    return {"oracle_table": rows, "host": {"cpu_model": model, "cores_visible": len(os.sched_getaffinity(0)),
                                           "threads": threads}}


def batch_bench(args, torch, synth, tp) -> dict:
    """Batched form: every graph of the batch built and surveyed together,
    against the same graphs built and surveyed one launch sequence each.

    A step is tripoll_build_batch + tripoll_survey_batch + readback of all
    per-graph results.  The recorded (HIP graph) survey launch is timed
    separately by replays on the resident batch.  The one-graph loop
    (tripoll_build + tripoll_survey per graph, synchronous) runs on every
    k-th graph; its total is that sample's time times k, an unbiased
    estimate of the loop over all graphs, and the sampled graphs' results
    must equal their blocks of the batch result."""
    w = synth.workload(4)
    ex = w.extra
    G = args.graphs or ex["n_graphs"]
    specs = synth.batch_specs(G, scale_lo=ex["scale_lo"], scale_hi=ex["scale_hi"], ef_lo=ex["ef_lo"],
                              ef_hi=ex["ef_hi"])
    eoff, vcnt = synth.batch_offsets(specs)
    M, N = int(eoff[-1]), int(vcnt.sum())
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream
    log("batch of %d graphs: %d vertices, %d raw edges; generating on the device" % (G, N, M))
    t0 = time.perf_counter()
    d = synth.generate_batch_device(specs, torch)
    src, dst, ts, vlab = d["src"], d["dst"], d["ts"], d["vlab"]
    del d
    torch.cuda.synchronize()
    log("  generated in %.1f s" % (time.perf_counter() - t0))
    outputs = w.outputs
    spec = tp.make_spec(outputs=outputs, n_labels=w.n_labels)
    bw = tp.tripoll_batch_words(spec)
    out = torch.zeros(G * bw + tp.TP_BATCH_SCRATCH_WORDS, dtype=torch.int64, device="cuda")
    be, keep = tp.batch_edges(eoff, vcnt, src, dst, ts, vlab, device=True)
    plan = tune = None
    if args.tune:
        h = tp.tripoll_build_batch(be, sptr)
        try:
            r = tp.tripoll_tune(h, spec, sptr)
            tune, plan = tp.tune_dict(r), r.chosen
        finally:
            tp.tripoll_graph_free(h)
        log("tuned plan: %s" % tune)

    def step():
        h = tp.tripoll_build_batch(be, sptr)
        try:
            if plan is not None:
                tp.tripoll_set_plan(h, plan, sptr)
            st = tp.stats_dict(tp.tripoll_graph_stats(h))
            tp.tripoll_survey_batch(h, spec, out.data_ptr(), sptr)
            words = out.cpu().numpy().view(np.uint64)  # synchronises the stream
        finally:
            tp.tripoll_graph_free(h)
        return st, words

    for i in range(args.warmup):
        st, words = step()
        log("warmup %d: build %.1f ms" % (i, st["build_ms"]))
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    per = []
    for i in range(args.steps):
        s0 = time.perf_counter()
        st, words = step()
        per.append(time.perf_counter() - s0)
        log("step %d: %.1f ms (build %.1f)" % (i, per[-1] * 1e3, st["build_ms"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = wall * 1e3 / args.steps
    res = tp.batch_dicts(words, G, spec, w.n_labels)
    tri = sum(r["triangles"] for r in res)
    probes = sum(r["probes"] for r in res)

    # recorded launch on the resident batch
    h = tp.tripoll_build_batch(be, sptr)
    rec_ms = []
    try:
        if plan is not None:
            tp.tripoll_set_plan(h, plan, sptr)
        st = tp.stats_dict(tp.tripoll_graph_stats(h))
        rec = torch.zeros_like(out)
        with tp.Launch(tp.tripoll_survey_capture(h, spec, rec.data_ptr())) as L:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            for i in range(max(3, args.steps)):
                e0.record(stream)
                L.replay(sptr)
                e1.record(stream)
                torch.cuda.synchronize()
                rec_ms.append(e0.elapsed_time(e1))
        assert np.array_equal(rec.cpu().numpy().view(np.uint64), words), "recorded launch differs from eager"
    finally:
        tp.tripoll_graph_free(h)
    log("recorded survey: %s ms" % ["%.2f" % x for x in rec_ms])

    # one graph per launch sequence, on every k-th graph
    k = max(1, args.loop_stride)
    sample = list(range(0, G, k))
    log("one-graph loop on %d sampled graphs" % len(sample))
    loop_build = loop_survey = 0.0
    v0s = np.concatenate([[0], np.cumsum(vcnt.astype(np.int64))])
    torch.cuda.synchronize()
    for g in sample:
        e0, e1 = int(eoff[g]), int(eoff[g + 1])
        n = int(vcnt[g])
        if n == 0:
            continue
        el = tp.edge_list(n, src[e0:e1], dst[e0:e1], ts[e0:e1], vlab[int(v0s[g]):int(v0s[g + 1])], device=True)
        t0 = time.perf_counter()
        hg = tp.tripoll_build(el, sptr)
        t1 = time.perf_counter()
        try:
            r1 = tp.result_dict(tp.tripoll_survey(hg, spec, sptr), w.n_labels)
        finally:
            tp.tripoll_graph_free(hg)
        t2 = time.perf_counter()
        loop_build += t1 - t0
        loop_survey += t2 - t1
        assert r1["triangles"] == res[g]["triangles"], g
        assert np.array_equal(r1["close_hist"], res[g]["close_hist"]), g
    loop_total_est = (loop_build + loop_survey) * k

    return {
        "metric": METRIC,
        "value": tri / (ms_per_step * 1e-3),
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name if G == ex["n_graphs"] else "batch-%d" % G, "graphs": G,
                   "scale_range": [ex["scale_lo"], ex["scale_hi"]], "edge_factor_range": [ex["ef_lo"], ex["ef_hi"]],
                   "kinds": "R-MAT or Erdos-Renyi 50/50", "raw_edges": M, "vertices": N, "edges": st["n_edges"],
                   "outputs": list(outputs),
                   "step": "batch build + batch survey + readback of every graph's counters"},
        "result": {"triangles": tri, "wedge_checks": probes, "graphs_per_s": G / (ms_per_step * 1e-3)},
        "batch": {"build_ms": round(st["build_ms"], 2), "build_phase_ms": [round(x, 2) for x in st["phase_ms"]],
                  "recorded_survey_ms_p50": round(statistics.median(rec_ms), 3),
                  "recorded_survey_triangles_per_s": tri / (statistics.median(rec_ms) * 1e-3),
                  "tiles": st["class_tiles"], "tune": tune,
                  "work": batch_work(st, tri, statistics.median(rec_ms), meta=tuple(outputs) != ("count",))},
        "one_graph_loop": {"sampled_graphs": len(sample), "stride": k,
                           "build_s_est": round(loop_build * k, 3), "survey_s_est": round(loop_survey * k, 3),
                           "total_s_est": round(loop_total_est, 3),
                           "batched_speedup": round(loop_total_est / (ms_per_step * 1e-3), 2),
                           "survey_speedup_recorded": round(loop_survey * k / (statistics.median(rec_ms) * 1e-3),
                                                            2)},
    }


def fifo_latencies(arrivals, service):
    """Latencies of a single server taking requests one at a time in arrival
    order, with the given service times (seconds)."""
    free_at = 0.0
    lat = []
    for a, sv in zip(arrivals, service):
        start = max(a, free_at)
        free_at = start + sv
        lat.append(free_at - a)
    return lat


def served_bench(args, torch, synth, tp) -> dict:
    """Served form: a resident R-MAT graph (scale 28 by default) and a pool
    of resident small graphs (scales 16..20) answer Poisson request streams
    through the survey server (continuous batching).  Request kinds on the
    large graph: full closure histograms (tag 0), time windows [t0, t0 + w]
    with w log-uniform in [2^12, 2^31] (tag 1), label-predicate counts
    (tag 2); on the pool graphs (tag 3): the same kinds at random.  Latency
    is arrival to result in host memory, measured by the server.

    Baseline: the same arrivals served one request at a time.  The time
    alone of one request of every (graph, kind) class is measured with
    tripoll_survey on the same resident graph, and a first-come-first-served
    single queue over the same arrival times, with those service times,
    gives the serial latencies."""
    w = synth.workload(5, scale=args.scale)
    ex = w.extra
    gs = w.graph
    rng = np.random.default_rng(synth.MASTER_SEED + 5)
    L = w.n_labels
    sptr = torch.cuda.current_stream().cuda_stream
    srv = tp.Server(max_slots=args.slots, n_labels=L)
    try:
        log("generating %s: n=%d raw edges=%d" % (w.name, gs.n, gs.n_edges))
        t0 = time.perf_counter()
        g = synth.generate(gs)
        dev = [torch.from_numpy(g[k].view(np.int32) if g[k].dtype == np.uint32 else g[k]).to("cuda")
               for k in ("src", "dst", "ts", "vlab")]
        del g
        torch.cuda.synchronize()
        log("generated and uploaded in %.1f s; building the resident graph" % (time.perf_counter() - t0))
        t0 = time.perf_counter()
        big = srv.add_graph(gs.n, *dev)
        build_s = time.perf_counter() - t0
        del dev
        torch.cuda.empty_cache()
        bst = srv.graph_stats(big)
        log("resident: m=%d, wedge checks %d, %.1f GB, built in %.1f s" % (
            bst["n_edges"], bst["probes"], bst["device_bytes"] / 1e9, build_s))
        pool = []
        for k, sc in enumerate(range(ex["pool_scale_lo"], ex["pool_scale_hi"] + 1)):
            ps = synth.GraphSpec("rmat", sc, 16, synth.MASTER_SEED + 50 + k, ("uniform", 31), ("uniform", L))
            pg = synth.generate(ps)
            pdev = [torch.from_numpy(pg[x].view(np.int32) if pg[x].dtype == np.uint32 else pg[x]).to("cuda")
                    for x in ("src", "dst", "ts", "vlab")]
            pool.append(srv.add_graph(ps.n, *pdev))
            del pdev
        torch.cuda.synchronize()
        log("pool of %d graphs resident; hbm %.1f of %.1f GB" % (len(pool), srv.stats()["hbm_used"] / 1e9,
                                                                 srv.stats()["hbm_budget"] / 1e9))

        # the request stream
        n_tab = tp.table_size(L)

        def make_request(kind):
            if kind == 0:
                return dict(outputs=("count", "close_hist"))
            if kind == 1:
                width = int(2 ** (12 + 19 * rng.random()))
                lo = int(rng.integers(0, 1 << 31))
                return dict(outputs=("count", "close_hist"), window=(lo, min(lo + width, (1 << 32) - 1)))
            mask = [int(i) for i in np.nonzero(rng.random(n_tab) < 0.5)[0]]
            return dict(outputs=("count",), label_mask=mask)

        reqs = []  # (arrival s, graph, tag, spec)
        for rate, is_big in ((args.rate_big, True), (args.rate_small, False)):
            t = 0.0
            while rate > 0:
                t += rng.exponential(1.0 / rate)
                if t >= args.duration:
                    break
                kind = int(rng.integers(0, 3))
                gid = big if is_big else pool[int(rng.integers(0, len(pool)))]
                reqs.append((t, gid, kind if is_big else 3, make_request(kind)))
        reqs.sort(key=lambda r: r[0])
        log("%d requests over %.0f s (%d on the large graph)" % (len(reqs), args.duration,
                                                               sum(1 for r in reqs if r[1] == big)))
        tickets = []
        start = time.perf_counter()
        for at, gid, tag, spec in reqs:
            delay = at - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(gid, tag=tag, **spec))
        log("all submitted after %.1f s; draining" % (time.perf_counter() - start))
        results = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - start
        st = srv.stats()
        log("served: %s" % {k: st[k] for k in ("completed", "steps", "elapsed_s")})

        # serial baseline: the time alone of the first request of every
        # (graph, kind) class, measured on the same resident graph, stands
        # for the service time of every request of that class
        log("timing one request of each class alone")
        alone = {}
        for at, gid, tag, spec in reqs:
            key = (gid, tag if gid == big else ("w" if "window" in spec else "m" if "label_mask" in spec else "h"))
            if key in alone:
                continue
            h = srv.graph(gid)
            t1 = time.perf_counter()
            tp.tripoll_survey(h, tp.make_spec(n_labels=L, **spec), sptr)
            alone[key] = time.perf_counter() - t1
        service = [alone[(gid, tag if gid == big else ("w" if "window" in spec else "m" if "label_mask" in spec
                                                        else "h"))] for at, gid, tag, spec in reqs]
        lat_serial = fifo_latencies([r[0] for r in reqs], service)
        tags = {0: "large: closure histogram", 1: "large: time window", 2: "large: label predicate",
                3: "pool (scale %d-%d)" % (ex["pool_scale_lo"], ex["pool_scale_hi"])}
        per = {}
        for tg, name in tags.items():
            ser = [l for l, r in zip(lat_serial, reqs) if r[2] == tg]
            per[name] = {"requests": int(st["count"][tg]), "p50_ms": round(st["p50_ms"][tg], 2),
                         "p99_ms": round(st["p99_ms"][tg], 2),
                         "serial_p50_ms": round(float(np.percentile(ser, 50)) * 1e3, 2) if ser else None,
                         "serial_p99_ms": round(float(np.percentile(ser, 99)) * 1e3, 2) if ser else None}
        tri = st["triangles"]
        serial_span = max(lat_serial[i] + reqs[i][0] for i in range(len(reqs))) if reqs else 0.0
        out = {
            "metric": METRIC,
            "value": tri / st["elapsed_s"],
            "unit": "triangles/s",
            "n_gpus": 1,
            "steps": len(reqs),
            "warmup": 0,
            "ms_per_step": round(st["elapsed_s"] * 1e3 / max(1, len(reqs)), 3),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "u32",
            "data": "synthetic",
            "config": {"workload": w.name, "kind": gs.kind, "scale": gs.scale, "edge_factor": gs.edge_factor,
                       "timestamps": list(gs.ts), "labels": list(gs.labels), "edges": bst["n_edges"],
                       "pool_scales": [ex["pool_scale_lo"], ex["pool_scale_hi"]], "duration_s": args.duration,
                       "rate_big_per_s": args.rate_big, "rate_small_per_s": args.rate_small,
                       "slots": args.slots,
                       "step": "one served request (value: triangles surveyed per second of serving)"},
            "served": {"requests": len(reqs), "completed": int(st["completed"]), "device_steps": int(st["steps"]),
                       "elapsed_s": round(st["elapsed_s"], 3), "wall_s": round(wall, 3),
                       "requests_per_s": round(st["completed"] / st["elapsed_s"], 3),
                       "triangles": int(tri), "latency": per,
                       "hbm_used_gb": round(st["hbm_used"] / 1e9, 2)},
            "serial_baseline": {"kind": "same arrivals, one request at a time (FIFO) with each request's "
                                        "measured time alone",
                                "span_s": round(serial_span, 3),
                                "requests_per_s": round(len(reqs) / serial_span, 3) if serial_span else None,
                                "service_s_large": round(float(np.mean([sv for sv, r in zip(service, reqs)
                                                                       if r[1] == big] or [0])), 3),
                                "service_s_pool": round(float(np.mean([sv for sv, r in zip(service, reqs)
                                                                      if r[1] != big] or [0])), 4)},
            "graph_build_s": round(build_s, 2),
        }
        return out
    finally:
        srv.close()


def kind_bench(args, torch, synth, tp) -> dict:
    """One step = build + the chosen kind on workload 1-3's graph.  The
    roofline is that of the whole call after the build (every class, plus
    the participation post-pass or the enumeration's counting pass); its
    algorithmic bytes are the survey's plus the records written."""
    w = synth.workload(args.workload, scale=args.scale)
    gs = w.graph
    g = synth.generate(gs)
    dev = {k: torch.from_numpy(g[k]).to("cuda") for k in ("src", "dst", "ts", "vlab")}
    del g
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream
    el = tp.edge_list(gs.n, dev["src"], dev["dst"], dev["ts"], dev["vlab"], device=True)
    outputs = tuple(w.outputs) + (("max_edge", "degree_table") if args.kind == "ext" else ())
    # Algorithm 3's 1024 bins span the time range: 2^bits for uniform times,
    # 2^31 for bursty ones
    time_bits = gs.ts[1] if gs.ts[0] == "uniform" else 31
    shift = max(0, time_bits - 10)
    spec = tp.make_spec(outputs=outputs, n_labels=w.n_labels, spread_lt=w.spread_lt, max_edge_shift=shift)
    bufs = {}

    def run_kind(h, st):
        """Returns (triangles, records or counters written in bytes)."""
        if args.kind == "ext":
            r = tp.result_dict(tp.tripoll_survey(h, spec, sptr), w.n_labels)
            return r["triangles"], 0, r
        if args.kind == "maxe":
            # Algorithm 3's exact counting set: values and counts of at most m entries
            if "mv" not in bufs:
                bufs["mv"] = torch.empty(max(st["n_edges"], 1), dtype=torch.int32, device="cuda")
                bufs["mc"] = torch.empty(max(st["n_edges"], 1), dtype=torch.int64, device="cuda")
            nv = tp.tripoll_max_edge_counts(h, spec, bufs["mv"].data_ptr(), bufs["mc"].data_ptr(), st["n_edges"],
                                            sptr)
            tri = int(bufs["mc"][:nv].sum().item()) if nv else 0
            return tri, 12 * nv, None
        if args.kind == "participation":
            if "v" not in bufs:
                bufs["v"] = torch.empty(gs.n, dtype=torch.int64, device="cuda")
                bufs["e"] = torch.empty(max(st["n_edges"], 1), dtype=torch.int64, device="cuda")
            tri = tp.tripoll_participation(h, tp.make_spec(), bufs["v"].data_ptr(), bufs["e"].data_ptr(), sptr)
            return tri, 8 * (gs.n + st["n_edges"]), None
        cap = args.enum_capacity
        if "r" not in bufs:
            bufs["r"] = torch.empty(cap * 9, dtype=torch.int32, device="cuda")
        tp.tripoll_set_plan(h, tp.make_plan((0, 0, 0, 0), (args.enum_tile,) * 4), sptr)
        e, total, max_tile = tp.tripoll_enum_open(h, tp.make_spec(), sptr)
        try:
            got = 0
            while True:
                k = tp.tripoll_enum_next(e, bufs["r"].data_ptr(), cap, sptr)
                if k == 0:
                    break
                got += k
        finally:
            tp.tripoll_enum_close(e)
        assert got == total
        return total, 36 * total, None

    def step():
        h = tp.tripoll_build(el, sptr)
        try:
            st = tp.stats_dict(tp.tripoll_graph_stats(h))
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            tri, written, r = run_kind(h, st)
            b.record(stream)
            torch.cuda.synchronize()
            return st, tri, written, a.elapsed_time(b), r
        finally:
            tp.tripoll_graph_free(h)

    for _ in range(args.warmup):
        step()
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        per.append(step())
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    st, tri, written, _, r = per[-1]
    kind_ms = statistics.median(x[3] for x in per)
    hits = r["class_triangles"] if r is not None else [0] * 4
    alg = sum(algorithmic_bytes(st, c, True, hits[c]) for c in range(4)) + written
    achieved = alg / (kind_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": tri / (ms_per_step * 1e-3), "unit": "triangles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": w.name, "kind": args.kind, "scale": gs.scale, "raw_edges": gs.n_edges,
                   "vertices": gs.n, "edges": st["n_edges"], "outputs": list(outputs), "max_edge_shift": shift,
                   "enum_capacity": args.enum_capacity if args.kind == "enum" else None,
                   "enum_tile_records": args.enum_tile if args.kind == "enum" else None,
                   "step": "build + " + args.kind},
        "result": {"triangles": tri, "wedge_checks": st["probes"]},
        "kind_ms_p50": round(kind_ms, 3),
        "build_ms_p50": round(statistics.median(x[0]["build_ms"] for x in per), 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "the whole %s call (every class)" % args.kind, "algorithmic_bytes": int(alg),
                     "written_bytes": int(written)},
    }
    if r is not None:
        out["class_ms"] = [round(x, 3) for x in r["class_ms"]]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=3, choices=(1, 2, 3, 4, 5))
    ap.add_argument("--duration", type=float, default=60.0, help="workload 5: seconds of request arrivals")
    ap.add_argument("--rate-big", type=float, default=0.5, help="workload 5: requests/s on the large graph")
    ap.add_argument("--rate-small", type=float, default=20.0, help="workload 5: requests/s on the pool graphs")
    ap.add_argument("--slots", type=int, default=8, help="workload 5: request slots per resident graph")
    ap.add_argument("--graphs", type=int, default=None, help="batch size override (workload 4)")
    ap.add_argument("--loop-stride", type=int, default=10,
                    help="workload 4: time the one-graph-per-launch loop on every k-th graph")
    ap.add_argument("--scale", type=int, default=None, help="override the R-MAT scale (same recipe)")
    ap.add_argument("--count-only", action="store_true", help="survey the triangle count only")
    ap.add_argument("--kind", default="survey", choices=("survey", "ext", "participation", "enum", "maxe"),
                    help="workloads 1-3: what each step runs after the build: the survey (default), the survey "
                         "with Algorithm 3's max-edge bins and the degree table added, the per-vertex and "
                         "per-edge participation counts, the streamed enumeration of every triangle, or "
                         "Algorithm 3's exact counting set (maxe)")
    ap.add_argument("--enum-capacity", type=int, default=1 << 28, help="--kind enum: records per chunk")
    ap.add_argument("--enum-tile", type=int, default=256,
                    help="--kind enum: records per tile of the plan the enumeration runs with (small tiles keep "
                         "every chunk spread over many workgroups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the survey plan once on the first build; every step then re-cuts its tiles "
                         "with the chosen plan (inside the timed step)")
    ap.add_argument("--cpu-scale", type=int, default=21)
    ap.add_argument("--oracle-table", action="store_true",
                    help="time the oracle alone (no GPU): clean and survey per workload, one thread and all")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the survey runs on one GPU; --gpus %d is not supported "
              "(across GPUs it would shard by splitting the work prefix of the targets)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.oracle_table:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, len(os.sched_getaffinity(0)))
        print(json.dumps(oracle_table(threads)), flush=True)
        return

    import torch
    import synth
    from paper_2107_12330_amd import tripoll as tp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    if args.workload == 4:
        print(json.dumps(batch_bench(args, torch, synth, tp)), flush=True)
        return
    if args.workload == 5:
        print(json.dumps(served_bench(args, torch, synth, tp)), flush=True)
        return
    if args.kind != "survey":
        print(json.dumps(kind_bench(args, torch, synth, tp)), flush=True)
        return

    w = synth.workload(args.workload, scale=args.scale)
    gs = w.graph
    log("generating %s: n=%d raw edges=%d" % (w.name, gs.n, gs.n_edges))
    t0 = time.perf_counter()
    g = synth.generate(gs)
    log("generated in %.1f s; uploading" % (time.perf_counter() - t0))
    dev = {k: torch.from_numpy(g[k]).to("cuda") for k in ("src", "dst", "ts", "vlab")}
    torch.cuda.synchronize()
    del g
    outputs = ("count",) if args.count_only else w.outputs
    meta = not args.count_only
    spec = tp.make_spec(outputs=outputs, n_labels=w.n_labels, spread_lt=w.spread_lt)
    el = tp.edge_list(gs.n, dev["src"], dev["dst"], dev["ts"], dev["vlab"], device=True)

    if args.copy_calibration:
        # a plain copy of known size: 4 GiB read + 4 GiB written
        a = torch.empty(1 << 30, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written per copy" % (a.numel() * 4, b.numel() * 4))
        del a, b

    plan = None
    tune = None
    if args.tune:
        h = tp.tripoll_build(el, sptr)
        try:
            r = tp.tripoll_tune(h, spec, sptr)
            tune = tp.tune_dict(r)
            plan = r.chosen
        finally:
            tp.tripoll_graph_free(h)
        log("tuned plan: %s" % tune)

    def step():
        h = tp.tripoll_build(el, sptr)
        try:
            if plan is not None:
                tp.tripoll_set_plan(h, plan, sptr)
            st = tp.stats_dict(tp.tripoll_graph_stats(h))
            pl = tp.plan_dict(tp.tripoll_get_plan(h))
            res = tp.tripoll_survey(h, spec, sptr)
        finally:
            tp.tripoll_graph_free(h)
        st["plan"] = pl
        return st, tp.result_dict(res, w.n_labels)

    for i in range(args.warmup):
        st, r = step()
        log("warmup %d: build %.1f ms, survey %.1f ms, %d triangles" % (i, st["build_ms"], r["total_ms"],
                                                                      r["triangles"]))

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    per = []
    for i in range(args.steps):
        s0 = time.perf_counter()
        st, r = step()
        per.append((time.perf_counter() - s0, st, r))
        log("step %d: %.1f ms (build %.1f, survey %.1f kernel %.1f), %d triangles" % (
            i, per[-1][0] * 1e3, st["build_ms"], r["total_ms"], r["kernel_ms"], r["triangles"]))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)

    st, r = per[-1][1], per[-1][2]
    tri = r["triangles"]
    for _, _, rr in per:
        assert rr["triangles"] == tri
    ms_per_step = wall * 1e3 / args.steps
    survey_ms = [rr["total_ms"] for _, _, rr in per]
    kernel_ms = [rr["kernel_ms"] for _, _, rr in per]
    build_ms = [s["build_ms"] for _, s, _ in per]

    # dominant survey kernel
    cls_ms = [statistics.mean(rr["class_ms"][c] for _, _, rr in per) for c in range(4)]
    hits = r["class_triangles"]
    c = int(np.argmax(cls_ms))
    alg = algorithmic_bytes(st, c, meta, hits[c])
    loaded = loaded_bytes(st, c, meta)
    achieved = alg / (cls_ms[c] * 1e-3) / 1e9
    var = st["plan"]["variant"][c]
    key = kernel_key(c, var, meta)
    traffic = load_traffic(key, w.name)
    survey_alg = sum(algorithmic_bytes(st, k, meta, hits[k]) for k in range(4))
    survey_t = statistics.median(kernel_ms) * 1e-3
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "%s: class %s, %s" % (key, CLASS_NAMES[c], VARIANT_NAMES[resolve_variant(c, var)]),
                "kernel_ms": round(cls_ms[c], 3), "algorithmic_bytes": int(alg),
                "algorithmic_model": "4 B per wedge check + 4 B per hit + %d B per staged out-list entry + 8 B per "
                                     "in-edge record + 16 B per tile" % (9 if meta else 4),
                "wedge_checks": int(st["class_probes"][c]), "hits": int(hits[c]),
                "staged": int(st["class_staged"][c]), "records": int(st["class_records"][c]),
                "tiles": int(st["class_tiles"][c]),
                "traffic_frac": None if traffic is None else round(traffic / (cls_ms[c] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic_per_algorithmic_byte": None if traffic is None else round(traffic / alg, 3),
                "loaded_bytes": int(loaded),
                "loaded_frac": round(loaded / (cls_ms[c] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "survey_algorithmic_bytes": int(survey_alg),
                "survey_frac": round(survey_alg / survey_t / 1e9 / HBM_PEAK_GBS, 4)}

    out = {
        "metric": METRIC,
        "value": tri / (ms_per_step * 1e-3),
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "kind": gs.kind, "scale": gs.scale, "edge_factor": gs.edge_factor,
                   "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "timestamps": list(gs.ts), "labels": list(gs.labels),
                   "outputs": list(outputs), "spread_lt": w.spread_lt, "seed": gs.seed,
                   "raw_edges": gs.n_edges, "vertices": gs.n, "edges": st["n_edges"],
                   "step": "build (canonicalise, sort, dedup, order, orient, CSR, in-edge index, plan) + survey"},
        "result": {"triangles": tri, "wedges": st["wedges"], "wedge_checks": r["probes"],
                   "spread_count": r["spread_count"], "d_max": st["d_max"], "dplus_max": st["dplus_max"]},
        "survey": {
            "triangles_per_s": tri / (statistics.median(survey_ms) * 1e-3),
            "wedge_checks_per_s": r["probes"] / (statistics.median(survey_ms) * 1e-3),
            "survey_ms_p50": statistics.median(survey_ms),
            "survey_ms_p99": float(np.percentile(survey_ms, 99)),
            "kernel_ms_p50": statistics.median(kernel_ms),
            "class_ms": [round(x, 3) for x in cls_ms],
            "build_ms_p50": statistics.median(build_ms),
            "build_phase_ms": [round(x, 2) for x in st["phase_ms"]],
            "gpu_ms_per_step": round(gpu_ms / args.steps, 3),
            "plan": st["plan"],
            "tune": tune,
        },
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        # the host's CPU share for this GPU: OMP_NUM_THREADS when set, else the visible cores (at most 16)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, len(os.sched_getaffinity(0)))
        log("cpu baseline: oracle at scale %d on %d threads" % (args.cpu_scale, threads))
        out["cpu_baseline"] = cpu_baseline(args.cpu_scale, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
