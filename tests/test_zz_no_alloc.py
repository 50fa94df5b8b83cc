"""The survey entry point that allocates nothing (tripoll_survey_noalloc):
its result words live in a static device array, so the library's allocator
and torch's see no new memory, and every counter equals tripoll_survey's on
the same graph and spec, on two calls in a row, the second on a smaller
graph."""
import sys

import numpy as np
import pytest

import synth
from paper_2107_12330_amd import tripoll as tp

pytestmark = pytest.mark.gpu

ALL_OUT = ("count", "close_hist", "label_table", "spread_count", "open_close")
KEYS = ("triangles", "spread_count", "probes", "close_hist", "label_table", "open_close", "max_edge",
        "degree_table", "directed", "class_triangles")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_graph(torch, spec):
    g = synth.generate(spec)
    dev = [torch.from_numpy(g[k]).cuda() for k in ("src", "dst", "ts", "vlab")]
    return g["n"], dev


def test_noalloc_equals_survey_on_two_calls():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    big = synth.GraphSpec("rmat", 17, 16, synth.MASTER_SEED + 701, ("uniform", 24), ("uniform", 8))
    small = synth.GraphSpec("rmat", 11, 8, synth.MASTER_SEED + 702, ("uniform", 20), ("uniform", 8))
    specs = [tp.make_spec(outputs=ALL_OUT, n_labels=8, spread_lt=1 << 14),
             tp.make_spec(outputs=("count", "close_hist", "max_edge", "degree_table"), n_labels=8,
                          max_edge_shift=14, window=(1 << 10, 3 << 22), label_mask=list(range(0, 120, 3)))]
    graphs = []
    for gs in (big, small):
        n, dev = device_graph(torch, gs)
        graphs.append(tp.build_graph(n, *dev, stream=stream))
    torch.cuda.synchronize()
    for k, (G, gs) in enumerate(zip(graphs, (big, small))):
        for j, spec in enumerate(specs):
            want = tp.result_dict(tp.tripoll_survey(G.handle, spec, stream), 8)
            tp.tripoll_trim()
            cached = tp.tripoll_cached_bytes()
            torch_bytes = torch.cuda.memory_allocated()
            say("call %d: scale %d, spec %d" % (k, gs.scale, j))
            got = tp.result_dict(tp.tripoll_survey_noalloc(G.handle, spec, stream), 8)
            assert tp.tripoll_cached_bytes() == cached == 0
            assert torch.cuda.memory_allocated() == torch_bytes
            for key in KEYS:
                assert np.array_equal(np.asarray(got[key]), np.asarray(want[key])), (k, j, key)
            assert sum(got["class_triangles"]) == got["triangles"]
            if j == 0:
                assert got["triangles"] > 0
    for G in graphs:
        G.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    torch.cuda.set_device(0)
    with pytest.raises(tp.TripollError) as e:
        tp.tripoll_survey_noalloc(None, tp.make_spec())
    assert e.value.status == tp.TP_ERR_INVALID
