"""GPU parity: the HIP survey against the CPU oracle, bit for bit.

All counters are integers, so the bar is exact equality of every counter.
Inputs are the seeded synthetic workloads; the oracle runs on the same bytes.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2107_12330_amd import tripoll as tp
from tests import graphs

pytestmark = pytest.mark.gpu

ALL_OUT = ("count", "close_hist", "label_table", "spread_count", "open_close")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def upload(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_build(torch, n, src, dst, ts, vlab, tie=tp.TP_TIE_MIX, device=True):
    if device:
        args = [upload(torch, x) if x is not None else None for x in (src, dst, ts, vlab)]
    else:
        args = [np.ascontiguousarray(x) if x is not None else None for x in (src, dst, ts, vlab)]
    return tp.build_graph(n, *args, tie=tie, stream=torch.cuda.current_stream().cuda_stream)


def gpu_survey(torch, G, **kw):
    return tp.survey(G, stream=torch.cuda.current_stream().cuda_stream, **kw)


def assert_same(got, ref, keys=("triangles", "close_hist", "label_table", "spread_count", "open_close")):
    for k in keys:
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        assert a.shape == b.shape and np.array_equal(a, b), (k, a, b)


def check_graph(torch, n, src, dst, ts, vlab, n_labels, spread_lt=1 << 16, outputs=ALL_OUT, tie=tp.TP_TIE_MIX,
                strategies=(tp.TP_STRAT_AUTO,), device=True, **kw):
    ref = oracle.survey(n, src, dst, ts, vlab, outputs=outputs, n_labels=n_labels, spread_lt=spread_lt, **kw)
    with gpu_build(torch, n, src, dst, ts, vlab, tie=tie, device=device) as G:
        st = G.stats()
        assert st["n_edges"] == ref["m"]
        for strat in strategies:
            got = gpu_survey(torch, G, outputs=outputs, n_labels=n_labels, spread_lt=spread_lt, strategy=strat, **kw)
            assert_same(got, ref)
            assert got["probes"] == st["probes"]
    return ref, st


# ---------------------------------------------------------------- small cases

def test_hand_worked_fixture(torch_cuda):
    import json, os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tiny_hand.json")))
    e = np.array(fx["edges"], np.uint32)
    say("hand fixture")
    ref, _ = check_graph(torch_cuda, fx["n"], e[:, 0], e[:, 1], e[:, 2], np.array(fx["labels"], np.uint8), 4,
                         strategies=(0, 1))
    assert ref["triangles"] == fx["expect"]["triangles"]


@pytest.mark.parametrize("n", [3, 4, 17, 100])
def test_complete_graphs(torch_cuda, n):
    u, v = zip(*itertools.combinations(range(n), 2))
    src, dst = np.array(u, np.uint32), np.array(v, np.uint32)
    ts = (np.arange(len(src)) * 7919 % 100000).astype(np.uint32)
    vlab = (np.arange(n) % 4).astype(np.uint8)
    say("K_%d" % n)
    ref, st = check_graph(torch_cuda, n, src, dst, ts, vlab, 4, strategies=(0, 1, 2))
    assert ref["triangles"] == math.comb(n, 3)


def test_huge_target_class(torch_cuda):
    # K_5000: d+ reaches 4999 > 3276, so the top targets are huge (surveyed
    # in two pieces of Adj+(q))
    n = 5000
    iu = np.triu_indices(n, 1)
    src, dst = iu[0].astype(np.uint32), iu[1].astype(np.uint32)
    rng = np.random.default_rng(0)
    ts = rng.integers(0, 1 << 20, len(src)).astype(np.uint32)
    vlab = rng.integers(0, 4, n).astype(np.uint8)
    say("K_5000")
    with gpu_build(torch_cuda, n, src, dst, ts, vlab) as G:
        st = G.stats()
        assert st["dplus_max"] == n - 1
        got = gpu_survey(torch_cuda, G, outputs=("count", "close_hist", "label_table"), n_labels=4)
        # every output over 16 labels: the counters leave too little LDS for
        # the doubled hit ring, so the pieces kernel takes the plain one
        wide = gpu_survey(torch_cuda, G, outputs=ALL_OUT, n_labels=16, spread_lt=1 << 30)
    assert got["triangles"] == math.comb(n, 3)
    assert int(got["close_hist"].sum()) == math.comb(n, 3)
    assert wide["triangles"] == got["triangles"] and np.array_equal(wide["close_hist"], got["close_hist"])
    assert int(np.asarray(wide["open_close"]).sum()) == math.comb(n, 3) and wide["spread_count"] == math.comb(n, 3)
    # the colex index of a label multiset does not depend on the label count
    assert np.array_equal(np.asarray(wide["label_table"])[:20], np.asarray(got["label_table"])[:20])
    assert not np.asarray(wide["label_table"])[20:].any()
    # label table of K_n from class sizes
    sizes = np.bincount(vlab, minlength=4)
    from tests.brute import colex_multisets
    idx = colex_multisets(4)
    for (a, b, c), i in idx.items():
        if a == b == c:
            e = math.comb(int(sizes[a]), 3)
        elif a == b:
            e = math.comb(int(sizes[a]), 2) * int(sizes[c])
        elif b == c:
            e = int(sizes[a]) * math.comb(int(sizes[b]), 2)
        else:
            e = int(sizes[a]) * int(sizes[b]) * int(sizes[c])
        assert int(got["label_table"][i]) == e


def test_doubled_and_plain_hit_rings_agree(torch_cuda):
    # K_1200 with 16 label values: small-class and large-class targets.  With
    # the count and closure histogram, the large class's 1024-thread kernel
    # queues its hits in the doubled ring.  With every output over 16 labels
    # its counters (an 816-entry label table, the 1024-word open/close
    # histogram, an 8 KB label lookup) leave too little LDS for that ring, so
    # it takes the plain one.  Both surveys must agree, and every output must
    # match its closed form.
    n = 1200
    i, j = np.triu_indices(n, 1)
    rng = np.random.default_rng(1200)
    ts = rng.integers(0, 1 << 24, len(i)).astype(np.uint32)
    vlab = rng.integers(0, 16, n).astype(np.uint8)
    say("K_1200, 16 labels")
    with gpu_build(torch_cuda, n, i.astype(np.uint32), j.astype(np.uint32), ts, vlab) as G:
        st = G.stats()
        assert st["dplus_max"] == n - 1 and st["class_tiles"][1] > 0 and st["class_tiles"][2] > 0
        a = gpu_survey(torch_cuda, G, outputs=("count", "close_hist"), n_labels=16)
        b = gpu_survey(torch_cuda, G, outputs=ALL_OUT, n_labels=16, spread_lt=1 << 30)
    tri = math.comb(n, 3)
    assert a["triangles"] == b["triangles"] == tri
    assert np.array_equal(a["close_hist"], b["close_hist"]) and int(a["close_hist"].sum()) == tri
    assert int(np.asarray(b["open_close"]).sum()) == tri
    # spread below 2^30 > every time difference: every triangle
    assert b["spread_count"] == tri
    sizes = np.bincount(vlab, minlength=16)
    from tests.brute import colex_multisets
    for (x, y, z), k in colex_multisets(16).items():
        if x == y == z:
            e = math.comb(int(sizes[x]), 3)
        elif x == y:
            e = math.comb(int(sizes[x]), 2) * int(sizes[z])
        elif y == z:
            e = int(sizes[x]) * math.comb(int(sizes[y]), 2)
        else:
            e = int(sizes[x]) * int(sizes[y]) * int(sizes[z])
        assert int(b["label_table"][k]) == e


def test_huge_targets_random_dense(torch_cuda):
    # the huge targets' out-lists are surveyed in pieces and every record's
    # candidates are cut at the pieces' rank bounds, at irregular places:
    # bit-exact on every output, the extended form too, with the HBM search
    # beside the default
    n, src, dst, ts, vlab = graphs.huge_targets(4242)
    ext = ALL_OUT + ("max_edge", "degree_table")
    say("huge targets", n, len(src))
    ref = oracle.survey(n, src, dst, ts, vlab, outputs=ext, n_labels=5, spread_lt=1 << 16, max_edge_shift=12)
    with gpu_build(torch_cuda, n, src, dst, ts, vlab) as G:
        st = G.stats()
        say("d+ max", st["dplus_max"], "huge tiles", st["class_tiles"][3])
        assert st["dplus_max"] > 3276 and st["class_tiles"][3] > 0
        for strat in (0, 1):
            got = gpu_survey(torch_cuda, G, outputs=ALL_OUT, n_labels=5, spread_lt=1 << 16, strategy=strat)
            assert_same(got, ref)
            assert got["probes"] == st["probes"]
        got = gpu_survey(torch_cuda, G, outputs=ext, n_labels=5, spread_lt=1 << 16, max_edge_shift=12)
        assert_same(got, ref, keys=("triangles", "close_hist", "label_table", "spread_count", "open_close",
                                    "max_edge", "degree_table"))
        # tiles of at most 16 records: many more tiles per piece
        tp.tripoll_set_plan(G.handle, tp.make_plan((0, 0, 0, 0), (1024, 1024, 1024, 16)),
                            torch_cuda.cuda.current_stream().cuda_stream)
        got = gpu_survey(torch_cuda, G, outputs=ALL_OUT, n_labels=5, spread_lt=1 << 16)
        assert_same(got, ref)


def test_zero_triangle_and_degenerate_graphs(torch_cuda):
    T = torch_cuda
    say("degenerate")
    # star, K_{a,b}
    star = np.arange(1, 300, dtype=np.uint32)
    with gpu_build(T, 300, np.zeros(299, np.uint32), star, None, None) as G:
        assert gpu_survey(T, G)["triangles"] == 0
        assert G.stats()["wedges"] == 0
    a, b = np.meshgrid(np.arange(20), np.arange(20, 45))
    with gpu_build(T, 45, a.ravel().astype(np.uint32), b.ravel().astype(np.uint32), None, None) as G:
        assert gpu_survey(T, G)["triangles"] == 0
    # only self-loops
    loops = np.arange(10, dtype=np.uint32)
    with gpu_build(T, 10, loops, loops, None, None) as G:
        st = G.stats()
        assert st["n_edges"] == 0 and st["n_self_loops"] == 10
        assert gpu_survey(T, G)["triangles"] == 0
    # no edges at all, on the host
    e = np.zeros(0, np.uint32)
    with gpu_build(T, 5, e, e, None, None, device=False) as G:
        assert G.stats()["n_edges"] == 0
        r = gpu_survey(T, G, outputs=ALL_OUT)
        assert r["triangles"] == 0 and r["close_hist"].sum() == 0
    # one vertex
    with gpu_build(T, 1, np.zeros(3, np.uint32), np.zeros(3, np.uint32), None, None) as G:
        assert gpu_survey(T, G)["triangles"] == 0


def test_invalid_inputs(torch_cuda):
    T = torch_cuda
    say("invalid")
    with pytest.raises(tp.TripollError) as ei:
        gpu_build(T, 10, np.array([1, 10], np.uint32), np.array([2, 3], np.uint32), None, None)
    assert ei.value.status == tp.TP_ERR_INVALID
    src = np.array([0, 1, 2], np.uint32)
    dst = np.array([1, 2, 0], np.uint32)
    with gpu_build(T, 3, src, dst, None, np.array([0, 1, 9], np.uint8)) as G:
        with pytest.raises(tp.TripollError):
            gpu_survey(T, G, outputs=("label_table",), n_labels=4)
        with pytest.raises(tp.TripollError):
            gpu_survey(T, G, outputs=("count",), window=(5, 4))
        assert gpu_survey(T, G, outputs=("label_table",), n_labels=10)["triangles"] == 1


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_against_oracle(torch_cuda, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(20, 3000))
    M = int(rng.integers(n, 40 * n))
    L = int(rng.integers(1, 17))
    src = rng.integers(0, n, M).astype(np.uint32)
    dst = rng.integers(0, n, M).astype(np.uint32)
    # a few dense clusters give triangles and a mixed d+ distribution
    hub = rng.integers(0, n, M // 4).astype(np.uint32) % max(1, n // 10)
    src[: M // 4] = hub
    ts = rng.integers(0, 1 << int(rng.integers(1, 33)), M, dtype=np.uint64).astype(np.uint32)
    vlab = rng.integers(0, L, n).astype(np.uint8)
    say("random seed", seed, n, M, L)
    check_graph(torch_cuda, n, src, dst, ts, vlab, L, spread_lt=int(rng.integers(0, 1 << 20)),
                strategies=(0, 1, 2), device=bool(seed % 2))


def test_filters_against_oracle(torch_cuda):
    w = synth.workload(1)
    g = synth.generate(w.graph)
    say("filters")
    for kw in [dict(window=(1 << 18, 3 << 18)), dict(window=(0, (1 << 32) - 1)), dict(window=(7, 7)),
               dict(label_mask=[0, 5, 19]), dict(label_mask=[5], window=(0, 1 << 19))]:
        check_graph(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 4, **kw)


# ---------------------------------------------------------------- the workloads

def test_workload1_scale12(torch_cuda):
    w = synth.workload(1)
    g = synth.generate(w.graph)
    say("workload 1")
    ref, st = check_graph(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 4,
                          strategies=(0, 1, 2), tie=tp.TP_TIE_MIX)
    assert ref["triangles"] > 100000


def test_tie_hash_invariance_and_wedges(torch_cuda):
    w = synth.workload(1, scale=14)
    g = synth.generate(w.graph)
    say("tie hash")
    ref = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], outputs=ALL_OUT, n_labels=4,
                        spread_lt=1 << 16)
    for tie in (tp.TP_TIE_MIX, tp.TP_TIE_ID):
        with gpu_build(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], tie=tie) as G:
            got = gpu_survey(torch_cuda, G, outputs=ALL_OUT, n_labels=4, spread_lt=1 << 16)
            assert_same(got, ref)
            if tie == tp.TP_TIE_ID:
                # identical orientation to the oracle's (degree, id) order
                assert G.stats()["wedges"] == ref["wedges"]


def test_workload2_reduced_scale(torch_cuda):
    w = synth.workload(2, scale=16)
    g = synth.generate(w.graph)
    say("workload 2 at scale 16")
    check_graph(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 8, outputs=w.outputs)


def test_workload3_reduced_scale(torch_cuda):
    w = synth.workload(3, scale=17)
    g = synth.generate(w.graph)
    say("workload 3 at scale 17")
    check_graph(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 4, outputs=w.outputs,
                spread_lt=w.spread_lt)


# ---------------------------------------------------------------- structure

def test_builder_invariants(torch_cuda):
    w = synth.workload(1, scale=13)
    g = synth.generate(w.graph)
    say("builder invariants")
    u, v, t = oracle.clean(g["n"], g["src"], g["dst"], g["ts"])
    with gpu_build(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"]) as G:
        st = G.stats()
        ex = tp.export(G)
    n, m = g["n"], len(u)
    rowptr, col = ex["rowptr"].astype(np.int64), ex["col"].astype(np.int64)
    assert st["n_edges"] == m and rowptr[-1] == m
    dplus = np.diff(rowptr)
    assert dplus.sum() == m
    # rows strictly increasing and every edge ascends in rank
    src_rank = np.repeat(np.arange(n), dplus)
    assert (col > src_rank).all()
    same_row = src_rank[1:] == src_rank[:-1]
    assert (col[1:][same_row] > col[:-1][same_row]).all()
    # degree order: rank_to_id sorted by degree
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    rid = ex["rank_to_id"].astype(np.int64)
    assert sorted(rid.tolist()) == list(range(n))
    assert (np.diff(deg[rid]) >= 0).all()
    # d+(v)^2 <= 2m
    assert (dplus.astype(np.float64) ** 2 <= 2 * m).all()
    assert st["dplus_max"] == dplus.max() and st["d_max"] == deg.max()
    assert st["wedges"] == int((dplus * (dplus - 1) // 2).sum())
    # the edge set with times equals the oracle's cleaned edge list
    a, b = rid[src_rank], rid[col]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    got = sorted(zip(lo.tolist(), hi.tolist(), ex["etime"].tolist()))
    assert got == sorted(zip(u.tolist(), v.tolist(), t.tolist()))
    # co-located labels
    assert np.array_equal(ex["tlabel"], g["vlab"][rid[col]])
    assert np.array_equal(ex["rank_label"], g["vlab"][rid])


def test_clique_csr_layout(torch_cuda):
    # A clique on 4200 vertices: every degree is 4199, so the order is the
    # tie hash and the rank-r row holds 4199 - r targets, rows of every
    # length up to 4199 in one graph.  The CSR (rows ascending), its times
    # and labels, and the counts (C(n,3) triangles and wedges, all closed)
    # must come out exact.
    n = 4200
    rng = np.random.default_rng(4200)
    i, j = np.triu_indices(n, 1)
    flip = rng.random(len(i)) < 0.5
    src = np.where(flip, j, i).astype(np.uint32)
    dst = np.where(flip, i, j).astype(np.uint32)
    ts = rng.integers(0, 1 << 30, len(i)).astype(np.uint32)
    vlab = rng.integers(0, 5, n).astype(np.uint8)
    say("clique rows", n, len(src))
    with gpu_build(torch_cuda, n, src, dst, ts, vlab) as G:
        st = G.stats()
        ex = tp.export(G)
        r = gpu_survey(torch_cuda, G, outputs=("count",))
    tri = n * (n - 1) * (n - 2) // 6
    assert st["dplus_max"] == n - 1 and st["wedges"] == tri and r["triangles"] == tri
    rowptr, col = ex["rowptr"].astype(np.int64), ex["col"].astype(np.int64)
    dplus = np.diff(rowptr)
    assert np.array_equal(dplus, np.arange(n - 1, -1, -1))
    src_rank = np.repeat(np.arange(n), dplus)
    same_row = src_rank[1:] == src_rank[:-1]
    assert (col > src_rank).all() and (col[1:][same_row] > col[:-1][same_row]).all()
    rid = ex["rank_to_id"].astype(np.int64)
    a, b = rid[src_rank], rid[col]
    got = np.minimum(a, b) * n + np.maximum(a, b)
    order = np.argsort(got)
    assert np.array_equal(got[order], i.astype(np.int64) * n + j)
    assert np.array_equal(ex["etime"][order], ts)
    assert np.array_equal(ex["tlabel"], vlab[rid[col]])


def test_enumeration_exactly_once(torch_cuda):
    T = torch_cuda
    w = synth.workload(1, scale=11)
    g = synth.generate(w.graph)
    say("enumeration")
    ref = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], outputs=("count",), n_labels=4,
                        records=True)
    with gpu_build(T, g["n"], g["src"], g["dst"], g["ts"], g["vlab"]) as G:
        cap = ref["triangles"] + 10
        buf = T.zeros(cap * 9, dtype=T.int32, device="cuda")
        nfound = tp.tripoll_enumerate(G.handle, buf.data_ptr(), cap, T.cuda.current_stream().cuda_stream)
        recs = buf.cpu().numpy().view(np.uint32).reshape(-1, 9)[:nfound]
    assert nfound == ref["triangles"]
    # canonical form: vertices sorted by id with each edge's time and each vertex's label
    canon = set()
    for a, b, c, tab, tac, tbc, la, lb, lc in recs.tolist():
        tm = {frozenset((a, b)): tab, frozenset((a, c)): tac, frozenset((b, c)): tbc}
        lab = {a: la, b: lb, c: lc}
        x, y, z = sorted((a, b, c))
        canon.add((x, y, z, tm[frozenset((x, y))], tm[frozenset((x, z))], tm[frozenset((y, z))],
                   lab[x], lab[y], lab[z]))
    assert len(canon) == nfound  # exactly once
    rr = ref["records"]
    want = set(zip(*(rr[f].tolist() for f in ("a", "b", "c", "t_ab", "t_ac", "t_bc", "l_a", "l_b", "l_c"))))
    assert canon == want


def test_async_matches_sync(torch_cuda):
    T = torch_cuda
    w = synth.workload(1)
    g = synth.generate(w.graph)
    say("async")
    s = T.cuda.Stream()
    with gpu_build(T, g["n"], g["src"], g["dst"], g["ts"], g["vlab"]) as G:
        spec = tp.make_spec(outputs=ALL_OUT, n_labels=4, spread_lt=1 << 16)
        sync = tp.result_dict(tp.tripoll_survey(G.handle, spec, T.cuda.current_stream().cuda_stream), 4)
        out = T.zeros(tp.TP_RESULT_WORDS, dtype=T.int64, device="cuda")
        with T.cuda.stream(s):
            for _ in range(3):
                tp.tripoll_survey_async(G.handle, spec, out.data_ptr(), s.cuda_stream)
        s.synchronize()
        got = tp.words_dict(out.cpu().numpy().view(np.uint64), 4)
    assert_same(got, sync)
