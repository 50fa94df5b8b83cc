"""GPU tests of the streamed enumeration: every triangle exactly once with its
six metadata items, across chunks that never overflow the caller's buffer,
against the oracle's triangle records."""
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


def canon(recs):
    """Records (a, b, c, t_ab, t_ac, t_bc, l_a, l_b, l_c) with the vertices in
    id order, each edge's time and each vertex's label carried along."""
    out = []
    for a, b, c, tab, tac, tbc, la, lb, lc in recs.tolist():
        tm = {frozenset((a, b)): tab, frozenset((a, c)): tac, frozenset((b, c)): tbc}
        lab = {a: la, b: lb, c: lc}
        x, y, z = sorted((a, b, c))
        out.append((x, y, z, tm[frozenset((x, y))], tm[frozenset((x, z))], tm[frozenset((y, z))],
                    lab[x], lab[y], lab[z]))
    return out


def oracle_records(n, src, dst, ts, vlab, window=None, label_mask=None, n_labels=4):
    r = oracle.survey(n, src, dst, ts, vlab, outputs=("count",), n_labels=n_labels, records=True)["records"]
    want = set()
    for x in zip(*(r[f].tolist() for f in ("a", "b", "c", "t_ab", "t_ac", "t_bc", "l_a", "l_b", "l_c"))):
        if window is not None and not all(window[0] <= t <= window[1] for t in x[3:6]):
            continue
        if label_mask is not None and oracle.msidx(*x[6:9]) not in label_mask:
            continue
        want.add(x)
    return want


def stream_all(torch, G, capacity, **spec_kw):
    e, total, max_tile = tp.tripoll_enum_open(G.handle, tp.make_spec(**spec_kw), stream(torch))
    try:
        cap = max(capacity, 1)
        buf = torch.full((cap * 9 + 9,), -1, dtype=torch.int32, device="cuda")
        got, chunks = [], 0
        while True:
            k = tp.tripoll_enum_next(e, buf.data_ptr(), capacity, stream(torch))
            if k == 0:
                break
            assert k <= capacity
            h = buf.cpu().numpy().view(np.uint32)
            got += canon(h[: k * 9].reshape(-1, 9))
            assert (h[k * 9:] == 0xFFFFFFFF).all()  # nothing past the chunk's records
            buf.fill_(-1)
            chunks += 1
        assert tp.tripoll_enum_next(e, buf.data_ptr(), capacity, stream(torch)) == 0
        return got, total, max_tile, chunks
    finally:
        tp.tripoll_enum_close(e)


def test_stream_workload1(torch_cuda):
    w = synth.workload(1)
    g = synth.generate(w.graph)
    want = oracle_records(g["n"], g["src"], g["dst"], g["ts"], g["vlab"])
    say("enum stream workload 1", len(want))
    with gpu_build(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"]) as G:
        e, total, max_tile = tp.tripoll_enum_open(G.handle, tp.make_spec(), stream(torch_cuda))
        tp.tripoll_enum_close(e)
        # one chunk, several, and the smallest capacity that always progresses
        for capacity in (len(want) + 5, len(want) // 7, max_tile):
            got, total, max_tile, chunks = stream_all(torch_cuda, G, capacity)
            say("capacity", capacity, "chunks", chunks, "largest tile", max_tile)
            assert total == len(want) and 0 < max_tile <= total
            assert len(got) == len(set(got)) == total  # exactly once
            assert set(got) == want
            if capacity < total:
                assert chunks > 1


def test_stream_with_filters(torch_cuda):
    w = synth.workload(1, scale=11)
    g = synth.generate(w.graph)
    say("enum stream filters")
    for kw in [dict(window=(1 << 18, 3 << 18)), dict(label_mask=[0, 5, 19]),
               dict(window=(0, 1 << 19), label_mask=[1, 2, 3, 4, 10])]:
        want = oracle_records(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], **kw)
        with gpu_build(torch_cuda, g["n"], g["src"], g["dst"], g["ts"], g["vlab"]) as G:
            got, total, _, _ = stream_all(torch_cuda, G, max(1, len(want) // 3 + 1), n_labels=4, **kw)
        assert total == len(want) and set(got) == want and len(got) == len(set(got))


def test_small_capacity_refused_then_resumed(torch_cuda):
    T = torch_cuda
    w = synth.workload(1, scale=10)
    g = synth.generate(w.graph)
    want = oracle_records(g["n"], g["src"], g["dst"], g["ts"], g["vlab"])
    say("enum stream refusal")
    with gpu_build(T, g["n"], g["src"], g["dst"], g["ts"], g["vlab"]) as G:
        e, total, max_tile = tp.tripoll_enum_open(G.handle, tp.make_spec(), stream(T))
        try:
            assert max_tile > 1
            buf = T.full((max_tile * 9,), -1, dtype=T.int32, device="cuda")
            got = []
            refused = 0
            while True:
                try:
                    k = tp.tripoll_enum_next(e, buf.data_ptr(), 1, stream(T))
                except tp.TripollError as err:
                    assert err.status == tp.TP_ERR_INVALID
                    refused += 1
                    assert (buf.cpu().numpy().view(np.uint32) == 0xFFFFFFFF).all()
                    k = tp.tripoll_enum_next(e, buf.data_ptr(), max_tile, stream(T))
                if k == 0:
                    break
                got += canon(buf.cpu().numpy().view(np.uint32)[: k * 9].reshape(-1, 9))
                buf.fill_(-1)
            assert refused > 0
            assert set(got) == want and len(got) == total
        finally:
            tp.tripoll_enum_close(e)


def test_stream_huge_targets_random(torch_cuda):
    # targets of d+ above 3276 whose records straddle the pieces of Adj+(q)
    # at irregular places; a label mask keeps the triangles labelled (0, 0, x)
    T = torch_cuda
    n, src, dst, ts, vlab = graphs.huge_targets(808)
    mask = [oracle.msidx(0, 0, c) for c in range(5)]
    want = oracle_records(n, src, dst, ts, vlab, label_mask=set(mask), n_labels=5)
    say("enum stream huge targets", len(want))
    with gpu_build(T, n, src, dst, ts, vlab) as G:
        assert G.stats()["class_tiles"][3] > 0
        got, total, _, chunks = stream_all(T, G, max(1, len(want) // 4 + 1), n_labels=5, label_mask=mask)
    assert total == len(want) and len(got) == len(set(got)) and set(got) == want and chunks >= 4


def test_stream_huge_targets_and_empty(torch_cuda):
    T = torch_cuda
    # K_3400: the top targets have d+ above the large class (HBM search); a
    # label mask keeps the triangles of the 12 vertices labelled 1
    n = 3400
    iu = np.triu_indices(n, 1)
    src, dst = iu[0].astype(np.uint32), iu[1].astype(np.uint32)
    ts = (src * 7 + dst).astype(np.uint32)
    vlab = (np.arange(n) < 12).astype(np.uint8)
    want = set()
    for a in range(12):
        for b in range(a + 1, 12):
            for c in range(b + 1, 12):
                want.add((a, b, c, a * 7 + b, a * 7 + c, b * 7 + c, 1, 1, 1))
    say("enum stream K_3400")
    mask = [oracle.msidx(1, 1, 1)]
    with gpu_build(T, n, src, dst, ts, vlab) as G:
        assert G.stats()["dplus_max"] == n - 1
        e, total, max_tile = tp.tripoll_enum_open(G.handle, tp.make_spec(n_labels=4, label_mask=mask), stream(T))
        tp.tripoll_enum_close(e)
        cap = max(max_tile, 40)
        got, total, max_tile, chunks = stream_all(T, G, cap, n_labels=4, label_mask=mask)
    assert total == 220 and chunks >= -(-220 // cap)
    assert len(got) == len(set(got)) == 220 and set(got) == want
    e0 = np.zeros(0, np.uint32)
    with gpu_build(T, 4, e0, e0, None, None) as G:
        got, total, max_tile, chunks = stream_all(T, G, 10)
        assert total == 0 and got == [] and chunks == 0
