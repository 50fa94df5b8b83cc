"""GPU parity of the batched workload at its full size: the 20,000-graph batch
(R-MAT or Erdos-Renyi 50/50, scales 6..16, edge factors 4..32, 4.35e9 raw
edges in all), built and surveyed as one, against the oracle's survey of
every graph alone (Algorithm 1 on each member; tests/golden/make_golden.py
--batch stores the oracle's values).

The batch is generated on the device by the device form of the input
generator; a first test checks that form byte for byte against the host
generator on a sample of the batch's graphs.
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from paper_2107_12330_amd import tripoll as tp

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "golden_batch_w4.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def batch_specs():
    ex = synth.workload(4).extra
    return synth.batch_specs(ex["n_graphs"], scale_lo=ex["scale_lo"], scale_hi=ex["scale_hi"], ef_lo=ex["ef_lo"],
                             ef_hi=ex["ef_hi"])


def test_device_generator_matches_host(torch_cuda):
    """The device batch generator writes the host generator's bytes."""
    torch = torch_cuda
    specs = batch_specs()
    top = [g for g, s in enumerate(specs) if s.scale == 16][:2]
    pick = [specs[g] for g in list(range(24)) + top]
    say("device generator: %d graphs" % len(pick))
    dev = synth.generate_batch_device(pick, torch)
    host = synth.generate_batch(pick)
    for k in ("src", "dst", "ts"):
        assert np.array_equal(dev[k].cpu().numpy().view(np.uint32), host[k]), k
    assert np.array_equal(dev["vlab"].cpu().numpy(), host["vlab"])
    assert np.array_equal(dev["edge_offsets"], host["edge_offsets"])


def test_full_batch_against_oracle(torch_cuda):
    """Every graph's triangle count, the sampled graphs' closure histograms
    and the sum of all histograms equal the oracle's; a recorded launch of
    the same survey replays to the eager result."""
    torch = torch_cuda
    if not os.path.exists(GOLDEN):
        pytest.skip("no stored oracle result for the batch")
    gold = json.load(open(GOLDEN))
    specs = batch_specs()
    G = len(specs)
    assert G == gold["n_graphs"]
    stream = torch.cuda.current_stream().cuda_stream
    say("generating %d graphs on the device" % G)
    d = synth.generate_batch_device(specs, torch)
    assert int(d["edge_offsets"][-1]) == gold["raw_edges"]
    say("building the batch: %d raw edges" % gold["raw_edges"])
    be, keep = tp.batch_edges(d["edge_offsets"], d["vertex_counts"], d["src"], d["dst"], d["ts"], d["vlab"],
                              device=True)
    h = tp.tripoll_build_batch(be, stream)
    with tp.Graph(h) as Gb:
        del d, be, keep
        torch.cuda.empty_cache()
        st = Gb.stats()
        assert st["n_edges"] == gold["edges"]
        assert tp.tripoll_graph_count(Gb.handle) == G
        spec = tp.make_spec(outputs=("count", "close_hist"), n_labels=gold["n_labels"])
        bw = tp.tripoll_batch_words(spec)
        out = torch.zeros(G * bw + tp.TP_BATCH_SCRATCH_WORDS, dtype=torch.int64, device="cuda")
        say("surveying")
        tp.tripoll_survey_batch(Gb.handle, spec, out.data_ptr(), stream)
        torch.cuda.synchronize()
        words = out.cpu().numpy().view(np.uint64).copy()
        got = tp.batch_dicts(words, G, spec, gold["n_labels"])
        tri = np.array([r["triangles"] for r in got], np.uint64)
        want = np.array(gold["triangles"], np.uint64)
        bad = np.nonzero(tri != want)[0]
        assert len(bad) == 0, "graphs %s differ" % bad[:10].tolist()
        assert int(tri.sum()) == gold["triangles_total"]
        total = np.zeros(32, np.uint64)
        for r in got:
            total += r["close_hist"]
        assert np.array_equal(total, np.array(gold["close_hist_total"], np.uint64))
        for g, hist in gold["close_hist_sample"].items():
            assert np.array_equal(got[int(g)]["close_hist"], np.array(hist, np.uint64)), g
        assert sum(r["probes"] for r in got) == st["probes"]
        say("recorded launch")
        rec = torch.zeros_like(out)
        with tp.Launch(tp.tripoll_survey_capture(Gb.handle, spec, rec.data_ptr())) as L:
            for rep in range(2):
                rec.fill_(-1)
                L.replay(stream)
                torch.cuda.synchronize()
                assert np.array_equal(rec.cpu().numpy().view(np.uint64), words), rep
