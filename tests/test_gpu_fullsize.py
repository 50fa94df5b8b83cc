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
