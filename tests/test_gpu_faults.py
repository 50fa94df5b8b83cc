"""Error paths forced from the host: every device allocation of a build, a
batch build and a survey is made to fail in turn (tripoll_fail_alloc_after);
each call must return TP_ERR_OOM and release everything it had taken, and the
library must work normally afterwards."""
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2107_12330_amd import tripoll as tp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    yield torch
    tp.tripoll_fail_alloc_after(0)


def fail_each_allocation(call, limit=400):
    """Run call() with its 1st, 2nd, ... device allocation failing until it
    succeeds; after every failure the library holds no more device memory
    than before.  Returns (allocations the call makes, its result)."""
    base = tp.tripoll_live_bytes()
    for n in range(1, limit):
        tp.tripoll_fail_alloc_after(n)
        try:
            out = call()
        except tp.TripollError as e:
            assert e.status == tp.TP_ERR_OOM, (n, str(e))
            assert "injected" in str(e)
            assert tp.tripoll_live_bytes() == base, n
            continue
        finally:
            pass
        tp.tripoll_fail_alloc_after(0)
        return n - 1, out
    raise AssertionError("the call kept failing")


def test_build_and_survey_fail_cleanly(torch_cuda):
    torch = torch_cuda
    w = synth.workload(1)
    g = synth.generate(w.graph)
    dev = {k: torch.from_numpy(g[k]).cuda() for k in ("src", "dst", "ts", "vlab")}
    stream = torch.cuda.current_stream().cuda_stream
    el = tp.edge_list(g["n"], dev["src"], dev["dst"], dev["ts"], dev["vlab"], device=True)
    n_build, h = fail_each_allocation(lambda: tp.tripoll_build(el, stream))
    say("the build makes %d device allocations" % n_build)
    assert n_build >= 5
    ref = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], outputs=w.outputs, n_labels=4)
    with tp.Graph(h) as G:
        spec = tp.make_spec(outputs=w.outputs, n_labels=4)
        n_survey, res = fail_each_allocation(lambda: tp.tripoll_survey(G.handle, spec, stream))
        say("the survey makes %d device allocations" % n_survey)
        assert n_survey >= 1
        got = tp.result_dict(res, 4)
        assert got["triangles"] == ref["triangles"]
        assert np.array_equal(got["close_hist"], ref["close_hist"])
        assert np.array_equal(got["label_table"], ref["label_table"])


def test_batch_build_fails_cleanly(torch_cuda):
    torch = torch_cuda
    specs = synth.batch_specs(12, master=synth.MASTER_SEED + 41, scale_lo=4, scale_hi=9)
    d = synth.generate_batch(specs)
    dev = [torch.from_numpy(d[k]).cuda() for k in ("src", "dst", "ts", "vlab")]
    stream = torch.cuda.current_stream().cuda_stream
    be, keep = tp.batch_edges(d["edge_offsets"], d["vertex_counts"], *dev, device=True)
    n_build, h = fail_each_allocation(lambda: tp.tripoll_build_batch(be, stream))
    say("the batch build makes %d device allocations" % n_build)
    with tp.Graph(h) as G:
        spec = tp.make_spec(outputs=("count", "close_hist"), n_labels=8)
        bw = tp.tripoll_batch_words(spec)
        out = torch.zeros(len(specs) * bw + tp.TP_BATCH_SCRATCH_WORDS, dtype=torch.int64, device="cuda")
        tp.tripoll_survey_batch(G.handle, spec, out.data_ptr(), stream)
        torch.cuda.synchronize()
        got = tp.batch_dicts(out.cpu().numpy().view(np.uint64), len(specs), spec, 8)
    e = d["edge_offsets"]
    v0 = np.concatenate([[0], np.cumsum(d["vertex_counts"].astype(np.int64))])
    for i, s in enumerate(specs):
        ref = oracle.survey(s.n, d["src"][e[i]:e[i + 1]], d["dst"][e[i]:e[i + 1]], d["ts"][e[i]:e[i + 1]],
                            d["vlab"][v0[i]:v0[i + 1]], outputs=("count", "close_hist"), n_labels=8)
        assert got[i]["triangles"] == ref["triangles"], i
        assert np.array_equal(got[i]["close_hist"], ref["close_hist"]), i
