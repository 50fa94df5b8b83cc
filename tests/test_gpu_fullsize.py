"""GPU parity at the workloads' full sizes, in the configuration bench.py
times (device-resident raw edges -> tripoll_build -> tripoll_survey).

Expected values are the oracle's, stored by tests/golden/make_golden.py (it
calls only the oracle and the input generator).  Properties that hold at any
size are checked beside them.
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from paper_2107_12330_amd import tripoll as tp

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL_OUT = ("count", "close_hist", "label_table", "spread_count", "open_close")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load_golden(workload, scale):
    path = os.path.join(GOLDEN, "golden_w%d_s%d.json" % (workload, scale))
    if not os.path.exists(path):
        pytest.skip("no stored oracle result for workload %d at scale %d" % (workload, scale))
    return json.load(open(path))


def device_graph(torch, w):
    g = synth.generate(w.graph)
    dev = {k: torch.from_numpy(g[k]).cuda() for k in ("src", "dst", "ts", "vlab")}
    torch.cuda.synchronize()
    return dev


def check_against_golden(got, gold):
    assert got["triangles"] == gold["triangles"]
    assert got["spread_count"] == gold["spread_count"]
    assert np.array_equal(got["close_hist"], np.array(gold["close_hist"], np.uint64))
    assert np.array_equal(got["label_table"], np.array(gold["label_table"], np.uint64))
    assert np.array_equal(got["open_close"].ravel(), np.array(gold["open_close"], np.uint64))


@pytest.mark.parametrize("workload,scale", [(2, 22), (3, 26)])
def test_full_size_against_oracle(workload, scale):
    import torch
    gold = load_golden(workload, scale)
    w = synth.workload(workload, scale=scale)
    say("workload %d at scale %d: generating" % (workload, scale))
    dev = device_graph(torch, w)
    stream = torch.cuda.current_stream().cuda_stream
    say("building")
    with tp.build_graph(w.graph.n, dev["src"], dev["dst"], dev["ts"], dev["vlab"], stream=stream) as G:
        st = G.stats()
        assert st["n_edges"] == gold["m"]
        say("surveying: %d edges, %d wedges" % (st["n_edges"], st["wedges"]))
        got = tp.survey(G, stream=stream, outputs=ALL_OUT, n_labels=gold["n_labels"], spread_lt=gold["spread_lt"])
        check_against_golden(got, gold)
        assert got["probes"] == st["probes"] == sum(st["class_probes"])
        assert sum(got["class_triangles"]) == gold["triangles"]
        assert all(t == 0 for t, k in zip(got["class_triangles"], st["class_tiles"]) if k == 0)
        # the count-only kernels find the same triangles
        c = tp.survey(G, stream=stream, outputs=("count",), n_labels=gold["n_labels"])
        assert c["triangles"] == gold["triangles"]
        # every reduction sums to the triangle count
        assert int(got["close_hist"].sum()) == int(got["label_table"].sum()) == gold["triangles"]
    del dev
    torch.cuda.empty_cache()


def test_scale22_invariances():
    """Tie-break hash and forced strategies do not change any counter."""
    import torch
    gold = load_golden(2, 22)
    w = synth.workload(2, scale=22)
    dev = device_graph(torch, w)
    stream = torch.cuda.current_stream().cuda_stream
    kw = dict(outputs=ALL_OUT, n_labels=gold["n_labels"], spread_lt=gold["spread_lt"])
    with tp.build_graph(w.graph.n, dev["src"], dev["dst"], dev["ts"], dev["vlab"], tie=tp.TP_TIE_ID,
                        stream=stream) as G:
        say("tie by id")
        check_against_golden(tp.survey(G, stream=stream, **kw), gold)
        # with ties broken by id the orientation is the oracle's
        assert G.stats()["wedges"] == gold["wedges_degree_id_order"]
        say("global search")
        check_against_golden(tp.survey(G, stream=stream, strategy=tp.TP_STRAT_GLOBAL_SEARCH, **kw), gold)
    del dev
    torch.cuda.empty_cache()


def test_scale22_extended_outputs():
    """Algorithm 3's bins, the degree table, the directed census and the
    participation counts at full size, against the oracle's stored values."""
    import torch
    from tests.golden.make_golden import participation_checksums
    path = os.path.join(GOLDEN, "golden_ext_w2_s22.json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle result for the extended outputs")
    gold = json.load(open(path))
    w = synth.workload(2, scale=22)
    dev = device_graph(torch, w)
    stream = torch.cuda.current_stream().cuda_stream
    n = w.graph.n
    with tp.build_graph(n, dev["src"], dev["dst"], dev["ts"], dev["vlab"], stream=stream, directed=True) as G:
        st = G.stats()
        assert st["n_edges"] == gold["m"]
        say("extended survey")
        got = tp.survey(G, stream=stream, outputs=("count", "max_edge", "degree_table", "directed"),
                        n_labels=gold["n_labels"], max_edge_shift=gold["max_edge_shift"])
        assert got["triangles"] == gold["triangles"]
        assert np.array_equal(got["max_edge"], np.array(gold["max_edge"], np.uint64))
        deg = np.zeros(tp.TP_DEGREE_MAX, np.uint64)
        for i, c in gold["degree_table"].items():
            deg[int(i)] = c
        assert np.array_equal(got["degree_table"], deg)
        assert np.array_equal(got["directed"], np.array(gold["directed"], np.uint64))
        say("participation")
        m = st["n_edges"]
        vc = torch.zeros(n, dtype=torch.int64, device="cuda")
        ec = torch.zeros(m, dtype=torch.int64, device="cuda")
        tri = tp.tripoll_participation(G.handle, tp.make_spec(), vc.data_ptr(), ec.data_ptr(), stream)
        assert tri == gold["triangles"]
        ex = tp.export(G)
        rid = ex["rank_to_id"].astype(np.int64)
        row = np.repeat(np.arange(n), np.diff(ex["rowptr"].astype(np.int64)))
        a, b = rid[row], rid[ex["col"].astype(np.int64)]
        got_p = participation_checksums(n, vc.cpu().numpy().view(np.uint64), np.minimum(a, b), np.maximum(a, b),
                                        ec.cpu().numpy().view(np.uint64))
        assert got_p == gold["participation"]
    del dev
    torch.cuda.empty_cache()
