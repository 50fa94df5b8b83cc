"""GPU parity of the local participation counts (triangles at every vertex
and at every edge) against the CPU oracle, bit for bit, with and without the
prefilters, on every search variant."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2107_12330_amd import tripoll as tp
from tests import graphs

pytestmark = pytest.mark.gpu


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


def gpu_build(torch, n, src, dst, ts, vlab):
    args = [torch.from_numpy(np.ascontiguousarray(x)).cuda() if x is not None else None
            for x in (src, dst, ts, vlab)]
    return tp.build_graph(n, *args, stream=stream(torch))


def gpu_participation(torch, G, **spec_kw):
    """(vertex counts by id, {(lo id, hi id): count}, triangles)."""
    st = G.stats()
    n, m = st["n_vertices"], st["n_edges"]
    vc = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    ec = torch.zeros(max(m, 1), dtype=torch.int64, device="cuda")
    tri = tp.tripoll_participation(G.handle, tp.make_spec(**spec_kw), vc.data_ptr(), ec.data_ptr(), stream(torch))
    v = vc.cpu().numpy().view(np.uint64)[:n]
    e = ec.cpu().numpy().view(np.uint64)[:m]
    ex = tp.export(G)
    rid = ex["rank_to_id"].astype(np.int64)
    row = np.repeat(np.arange(n), np.diff(ex["rowptr"].astype(np.int64)))
    a, b = rid[row], rid[ex["col"].astype(np.int64)]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    return v, dict(zip(zip(lo.tolist(), hi.tolist()), e.tolist())), tri


def check(torch, n, src, dst, ts, vlab, n_labels=4, strategies=(0,), **kw):
    ref_v, (u, v, t, ref_e) = oracle.participation(n, src, dst, ts, vlab, n_labels=n_labels, **kw)
    want_e = dict(zip(zip(u.tolist(), v.tolist()), ref_e.tolist()))
    with gpu_build(torch, n, src, dst, ts, vlab) as G:
        for strat in strategies:
            gv, ge, tri = gpu_participation(torch, G, n_labels=n_labels, strategy=strat, **kw)
            assert np.array_equal(gv, ref_v), np.nonzero(gv != ref_v)[0][:8]
            assert ge == want_e
            assert 3 * tri == int(ref_v.sum()) == int(ref_e.sum())
    return ref_v, ref_e


def random_graph(rng, n, M, L, tbits):
    src = rng.integers(0, n, M).astype(np.uint32)
    dst = rng.integers(0, n, M).astype(np.uint32)
    hub = rng.integers(0, n, M // 4).astype(np.uint32) % max(1, n // 10)
    src[: M // 4] = hub
    ts = rng.integers(0, 1 << tbits, M, dtype=np.uint64).astype(np.uint32)
    vlab = rng.integers(0, L, n).astype(np.uint8)
    return src, dst, ts, vlab


@pytest.mark.parametrize("seed", range(5))
def test_random_graphs(torch_cuda, seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(20, 4000))
    M = int(rng.integers(n, 40 * n))
    L = int(rng.integers(1, 17))
    src, dst, ts, vlab = random_graph(rng, n, M, L, 20)
    say("participation random", seed, n, M, L)
    check(torch_cuda, n, src, dst, ts, vlab, L, strategies=(0, 1, 2))


def test_filters(torch_cuda):
    w = synth.workload(1)
    g = synth.generate(w.graph)
    say("participation filters")
    for kw in [dict(window=(1 << 18, 3 << 18)), dict(label_mask=[0, 5, 19]),
               dict(window=(0, 1 << 19), label_mask=[3, 4, 9, 12])]:
        check(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], 4, strategies=(0, 1), **kw)


def test_rmat_reduced_workloads(torch_cuda):
    for wl, scale, L in [(3, 15, 4), (2, 14, 8)]:
        w = synth.workload(wl, scale=scale)
        g = synth.generate(w.graph)
        say("participation workload", wl, "scale", scale)
        v, e = check(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"], L)
        assert v.sum() > 0


def test_complete_graph_huge_targets(torch_cuda):
    # K_4500 sends its top targets to the HBM search: every vertex is in
    # C(n-1, 2) triangles and every edge in n - 2
    n = 4500
    iu = np.triu_indices(n, 1)
    src, dst = iu[0].astype(np.uint32), iu[1].astype(np.uint32)
    say("participation K_4500")
    with gpu_build(torch_cuda, n, src, dst, None, None) as G:
        v, e, tri = gpu_participation(torch_cuda, G)
    assert tri == math.comb(n, 3)
    assert (v == math.comb(n - 1, 2)).all()
    assert len(e) == math.comb(n, 2) and set(e.values()) == {n - 2}


def test_huge_targets_random_dense(torch_cuda):
    # huge targets surveyed in pieces: the (q, r) counts of every piece's
    # table go back to the right CSR slots, the (p, q) counts add up over
    # the pieces
    n, src, dst, ts, vlab = graphs.huge_targets(77)
    say("participation huge targets", n, len(src))
    check(torch_cuda, n, src, dst, ts, vlab, 5, strategies=(0, 1))


def test_degenerate_and_null_outputs(torch_cuda):
    T = torch_cuda
    say("participation degenerate")
    e0 = np.zeros(0, np.uint32)
    with gpu_build(T, 5, e0, e0, None, None) as G:
        v, e, tri = gpu_participation(T, G)
        assert tri == 0 and v.sum() == 0 and not e
    star = np.arange(1, 100, dtype=np.uint32)
    with gpu_build(T, 100, np.zeros(99, np.uint32), star, None, None) as G:
        v, e, tri = gpu_participation(T, G)
        assert tri == 0 and v.sum() == 0 and sum(e.values()) == 0
    # a wheel on 6 spokes; either output may be omitted
    k = 6
    s = np.array([0] * k + list(range(1, k + 1)), np.uint32)
    d = np.array(list(range(1, k + 1)) + [i % k + 1 for i in range(1, k + 1)], np.uint32)
    with gpu_build(T, k + 1, s, d, None, None) as G:
        vc = T.zeros(k + 1, dtype=T.int64, device="cuda")
        assert tp.tripoll_participation(G.handle, tp.make_spec(), vc.data_ptr(), 0, stream(T)) == k
        v = vc.cpu().numpy()
        assert v[0] == k and (v[1:] == 2).all()
        assert tp.tripoll_participation(G.handle, tp.make_spec(), 0, 0, stream(T)) == k


def test_batch_of_two_triangles(torch_cuda):
    # two graphs, each one triangle: the union has two, every vertex and
    # every edge is in exactly one; without output arrays only the total
    T = torch_cuda
    src = np.array([0, 1, 0, 0, 1, 0], np.uint32)
    dst = np.array([1, 2, 2, 1, 2, 2], np.uint32)
    with tp.build_batch([0, 3, 6], [3, 3], src, dst, stream=stream(T)) as B:
        assert tp.tripoll_participation(B.handle, tp.make_spec(), 0, 0, stream(T)) == 2
        gv, ge, tri = gpu_participation(T, B)
        assert tri == 2
        assert gv.tolist() == [1] * 6
        assert ge == {(0, 1): 1, (0, 2): 1, (1, 2): 1, (3, 4): 1, (3, 5): 1, (4, 5): 1}


def test_batch_participation_per_graph(torch_cuda):
    """A batch handle counts the union of its graphs: every graph's slice of
    the vertex and edge counts equals the oracle's counts of that graph
    alone (ids offset by the graphs before it), with and without filters."""
    torch = torch_cuda
    specs = synth.batch_specs(14, master=synth.MASTER_SEED + 771, scale_lo=4, scale_hi=10)
    d = synth.generate_batch(specs)
    dev = [torch.from_numpy(d[k]).cuda() for k in ("src", "dst", "ts", "vlab")]
    e = d["edge_offsets"]
    voff = np.concatenate([[0], np.cumsum(d["vertex_counts"].astype(np.int64))])
    with tp.build_batch(d["edge_offsets"], d["vertex_counts"], *dev, stream=stream(torch)) as B:
        for kw in ({}, {"window": (1 << 17, 1 << 19)}, {"label_mask": {0, 3, 9, 17}}):
            say("batch participation %s" % kw)
            gv, ge, tri = gpu_participation(torch, B, n_labels=8, **kw)
            total = 0
            for g, sp in enumerate(specs):
                lo, hi = int(voff[g]), int(voff[g + 1])
                ref_v, (u, v, t, ref_e) = oracle.participation(
                    sp.n, d["src"][e[g]:e[g + 1]], d["dst"][e[g]:e[g + 1]], d["ts"][e[g]:e[g + 1]],
                    d["vlab"][lo:hi], n_labels=8, **kw)
                assert np.array_equal(gv[lo:hi], ref_v), g
                want = dict(zip(zip((u.astype(np.int64) + lo).tolist(), (v.astype(np.int64) + lo).tolist()),
                                ref_e.tolist()))
                got = {k: c for k, c in ge.items() if lo <= k[0] < hi}
                assert got == want, g
                total += int(ref_e.sum())
            assert 3 * tri == total == int(gv.sum())
