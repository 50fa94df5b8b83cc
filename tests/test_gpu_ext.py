"""GPU parity of the extended reductions against the CPU oracle, bit for bit:
Algorithm 3's largest-edge-time bins over triangles with pairwise distinct
vertex labels, and the degree-log triple table of the evaluation's metadata
experiment.  Also the documented refusals (batches, served requests, bad
arguments)."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2107_12330_amd import tripoll as tp

pytestmark = pytest.mark.gpu

EXT_OUT = ("count", "close_hist", "label_table", "spread_count", "open_close", "max_edge", "degree_table")
KEYS = ("triangles", "close_hist", "label_table", "spread_count", "open_close", "max_edge", "degree_table")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def stream(torch):
    return torch.cuda.current_stream().cuda_stream


def gpu_build(torch, n, src, dst, ts, vlab, tie=tp.TP_TIE_MIX):
    args = [torch.from_numpy(np.ascontiguousarray(x)).cuda() if x is not None else None
            for x in (src, dst, ts, vlab)]
    return tp.build_graph(n, *args, tie=tie, stream=stream(torch))


def assert_same(got, ref, keys=KEYS):
    for k in keys:
        a, b = np.asarray(got[k]).ravel(), np.asarray(ref[k]).ravel()
        assert a.shape == b.shape and np.array_equal(a, b), (k, np.nonzero(a != b)[0][:8])


def check(torch, n, src, dst, ts, vlab, n_labels, outputs=EXT_OUT, strategies=(tp.TP_STRAT_AUTO,), **kw):
    ref = oracle.survey(n, src, dst, ts, vlab, outputs=outputs, n_labels=n_labels, **kw)
    with gpu_build(torch, n, src, dst, ts, vlab) as G:
        st = G.stats()
        for strat in strategies:
            got = tp.survey(G, stream=stream(torch), outputs=outputs, n_labels=n_labels, strategy=strat, **kw)
            keys = [k for k in KEYS if k == "triangles" or k in outputs]
            assert_same(got, ref, keys)
            assert got["probes"] == st["probes"]
    return ref, st


def random_graph(rng, n, M, L, tbits):
    src = rng.integers(0, n, M).astype(np.uint32)
    dst = rng.integers(0, n, M).astype(np.uint32)
    hub = rng.integers(0, n, M // 4).astype(np.uint32) % max(1, n // 10)
    src[: M // 4] = hub
    ts = rng.integers(0, 1 << tbits, M, dtype=np.uint64).astype(np.uint32)
    vlab = rng.integers(0, L, n).astype(np.uint8)
    return src, dst, ts, vlab


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs(torch_cuda, seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(20, 4000))
    M = int(rng.integers(n, 40 * n))
    L = int(rng.integers(3, 17))
    tbits = int(rng.integers(1, 33))
    shift = int(rng.integers(0, 32))
    src, dst, ts, vlab = random_graph(rng, n, M, L, tbits)
    say("ext random", seed, n, M, L, tbits, shift)
    ref, _ = check(torch_cuda, n, src, dst, ts, vlab, L, strategies=(0, 1, 2), max_edge_shift=shift,
                   spread_lt=1 << 12)
    assert ref["degree_table"].sum() == ref["triangles"]


def test_single_outputs_and_filters(torch_cuda):
    rng = np.random.default_rng(77)
    n, L = 2500, 6
    src, dst, ts, vlab = random_graph(rng, n, 60000, L, 20)
    say("ext single outputs")
    for outputs in [("max_edge",), ("degree_table",), ("count", "max_edge", "degree_table")]:
        check(torch_cuda, n, src, dst, ts, vlab, L, outputs=outputs, max_edge_shift=10)
    for kw in [dict(window=(1 << 18, 3 << 18)), dict(label_mask=[1, 9, 30, 55]),
               dict(window=(0, (1 << 32) - 1), label_mask=list(range(0, 56, 3)))]:
        check(torch_cuda, n, src, dst, ts, vlab, L, outputs=("count", "max_edge", "degree_table"),
              max_edge_shift=8, **kw)


def test_rmat_workloads_reduced(torch_cuda):
    # scale-14 R-MAT with the scale-26 workload's bursty times (bins of 2^21
    # cover [0, 2^31)) and the scale-22 workload's Zipf labels
    w3 = synth.workload(3, scale=14)
    g = synth.generate(w3.graph)
    say("ext workload 3 at scale 14")
    ref, st = check(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 4, max_edge_shift=21,
                    strategies=(0, 1))
    # times are clamped to 2^31 - 1, whose bin is 1023
    assert ref["max_edge"].sum() > 0 and ref["max_edge"][:1024].sum() == ref["max_edge"].sum()
    w2 = synth.workload(2, scale=15)
    g = synth.generate(w2.graph)
    say("ext workload 2 at scale 15")
    check(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 8, max_edge_shift=20)


def test_huge_targets_complete_graph(torch_cuda):
    # K_4500: targets with d+ above the large class search Adj+(q) in HBM
    n = 4500
    iu = np.triu_indices(n, 1)
    src, dst = iu[0].astype(np.uint32), iu[1].astype(np.uint32)
    # the largest edge time of a triangle a<b<c is c: max(u, v) per edge
    ts = np.maximum(src, dst).astype(np.uint32)
    vlab = (np.arange(n) % 7).astype(np.uint8)
    say("ext K_4500")
    with gpu_build(torch_cuda, n, src, dst, ts, vlab) as G:
        assert G.stats()["dplus_max"] == n - 1
        got = tp.survey(G, stream=stream(torch_cuda), outputs=("count", "max_edge", "degree_table"), n_labels=7,
                        max_edge_shift=3)
    assert got["triangles"] == math.comb(n, 3)
    # every vertex has degree n-1
    b = (n - 2).bit_length()
    assert got["degree_table"][b * (b + 1) * (b + 2) // 6 + b * (b + 1) // 2 + b] == math.comb(n, 3)
    assert got["degree_table"].sum() == math.comb(n, 3)
    # closed form of Algorithm 3: for top vertex c, pairs a<b<c with three distinct residues mod 7
    cls = np.bincount(vlab, minlength=7)
    exp = np.zeros(1024, np.uint64)
    below = np.zeros(7, np.int64)
    for c in range(n):
        lc = int(vlab[c])
        others = [int(below[x]) for x in range(7) if x != lc]
        pairs = (sum(others) ** 2 - sum(o * o for o in others)) // 2
        exp[min(1023, c >> 3)] += pairs
        below[lc] += 1
    assert cls.sum() == n
    assert np.array_equal(got["max_edge"], exp)


def test_star_with_leaf_edges_overflows_tiny_tables(torch_cuda):
    # a hub of degree above 2^20: the degree table needs 22 bins, C(24,3) =
    # 2024 counters, which with every other output does not fit the per-wave
    # counters of the tiny class; that class then searches in HBM instead
    n = (1 << 20) + 1
    rng = np.random.default_rng(5)
    leaves = np.arange(1, n, dtype=np.uint32)
    a = rng.integers(1, n, 300000).astype(np.uint32)
    b = rng.integers(1, n, 300000).astype(np.uint32)
    src = np.concatenate([np.zeros(n - 1, np.uint32), a])
    dst = np.concatenate([leaves, b])
    ts = rng.integers(0, 1 << 24, len(src)).astype(np.uint32)
    vlab = rng.integers(0, 16, n).astype(np.uint8)
    say("ext star 2^20")
    ref, st = check(torch_cuda, n, src, dst, ts, vlab, 16, max_edge_shift=14)
    assert st["d_max"] >= 1 << 20
    assert ref["triangles"] >= 290000


def test_degenerate_graphs(torch_cuda):
    T = torch_cuda
    say("ext degenerate")
    e = np.zeros(0, np.uint32)
    with gpu_build(T, 5, e, e, None, None) as G:
        r = tp.survey(G, stream=stream(T), outputs=EXT_OUT, n_labels=4)
        assert r["triangles"] == 0 and r["max_edge"].sum() == 0 and r["degree_table"].sum() == 0
    # one triangle, labels 0, 1, 2 and times 5, 9, 700
    src = np.array([0, 1, 0], np.uint32)
    dst = np.array([1, 2, 2], np.uint32)
    ts = np.array([5, 9, 700], np.uint32)
    with gpu_build(T, 3, src, dst, ts, np.array([0, 1, 2], np.uint8)) as G:
        r = tp.survey(G, stream=stream(T), outputs=EXT_OUT, n_labels=4, max_edge_shift=2)
    assert r["triangles"] == 1 and r["max_edge"][700 >> 2] == 1 and r["max_edge"].sum() == 1
    assert r["degree_table"][oracle.msidx(1, 1, 1)] == 1  # three vertices of degree 2
    assert r["degree_table"].sum() == 1
    # a star has no triangle
    star = np.arange(1, 200, dtype=np.uint32)
    with gpu_build(T, 200, np.zeros(199, np.uint32), star, None, None) as G:
        r = tp.survey(G, stream=stream(T), outputs=EXT_OUT, n_labels=1)
        assert r["degree_table"].sum() == 0 and r["max_edge"].sum() == 0


def test_refusals(torch_cuda):
    T = torch_cuda
    say("ext refusals")
    src = np.array([0, 1, 0], np.uint32)
    dst = np.array([1, 2, 2], np.uint32)
    with gpu_build(T, 3, src, dst, None, None) as G:
        with pytest.raises(tp.TripollError) as ei:
            tp.survey(G, stream=stream(T), outputs=("max_edge",), max_edge_shift=32)
        assert ei.value.status == tp.TP_ERR_INVALID
        sp = tp.make_spec(outputs=("count",))
        sp.reserved = 1
        with pytest.raises(tp.TripollError) as ei:
            tp.tripoll_survey(G.handle, sp, stream(T))
        assert ei.value.status == tp.TP_ERR_INVALID
        # a single graph through the batch entry point: one block with its table
        spec = tp.make_spec(outputs=("degree_table",))
        out = T.zeros(tp.tripoll_batch_words(spec) + tp.TP_BATCH_SCRATCH_WORDS, dtype=T.int64, device="cuda")
        tp.tripoll_survey_batch(G.handle, spec, out.data_ptr(), stream(T))
        T.cuda.synchronize()
        blk = tp.batch_dicts(out.cpu().numpy().view(np.uint64), 1, spec, 4)[0]
        one = tp.survey(G, stream=stream(T), outputs=("degree_table",))
        assert blk["triangles"] == one["triangles"] == 1
        assert np.array_equal(blk["degree_table"], one["degree_table"])
    # a batch of two graphs: the union's degree table is refused outside the batch survey
    src2 = np.concatenate([src, src])
    dst2 = np.concatenate([dst, dst])
    with tp.build_batch([0, 3, 6], [3, 3], src2, dst2, stream=stream(T)) as B:
        with pytest.raises(tp.TripollError) as ei:
            tp.survey(B, stream=stream(T), outputs=("degree_table",))
        assert ei.value.status == tp.TP_ERR_UNSUPPORTED
        # the union's Algorithm 3 bins are those of its two triangles
        assert tp.survey(B, stream=stream(T), outputs=("max_edge",))["triangles"] == 2
    with tp.Server(max_slots=2, n_labels=4) as srv:
        gid = srv.add_graph(3, T.from_numpy(src).cuda(), T.from_numpy(dst).cuda())
        for outputs in [("max_edge",), ("degree_table",)]:
            r, _ = srv.wait(srv.submit(gid, outputs=outputs), timeout_us=60_000_000)
            assert r["triangles"] == 1 and r["max_edge" if "max_edge" in outputs else "degree_table"].sum() <= 1
