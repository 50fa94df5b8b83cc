"""GPU parity of every survey plan: each search variant of each target
class, at several tile caps, and the autotuner's choice, against the oracle.

The plan decides only how the work is cut and searched, so every counter
must stay identical to the oracle's under every plan.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2107_12330_amd import tripoll as tp

pytestmark = pytest.mark.gpu

OUT = ("count", "close_hist", "label_table", "spread_count", "open_close")
SPREAD = 1 << 14
V = tp


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch


def mixed_graph():
    """R-MAT scale 13 (tiny and small targets) with a planted K_900 on
    vertices 0..899 (targets of d+ up to 899: the large class)."""
    g = synth.generate(synth.GraphSpec("rmat", 13, 16, synth.MASTER_SEED + 77, ("uniform", 20), ("uniform", 4)))
    k = 900
    iu = np.triu_indices(k, 1)
    rng = np.random.default_rng(3)
    src = np.concatenate([g["src"], iu[0].astype(np.uint32)])
    dst = np.concatenate([g["dst"], iu[1].astype(np.uint32)])
    ts = np.concatenate([g["ts"], rng.integers(0, 1 << 20, len(iu[0])).astype(np.uint32)])
    return g["n"], src, dst, ts, g["vlab"]


@pytest.fixture(scope="module")
def mixed(torch_cuda):
    n, src, dst, ts, vlab = mixed_graph()
    say("oracle on the mixed graph")
    ref = oracle.survey(n, src, dst, ts, vlab, outputs=OUT, n_labels=4, spread_lt=SPREAD)
    dev = [torch_cuda.from_numpy(x).cuda() for x in (src, dst, ts, vlab)]
    return n, dev, ref


def check(got, ref):
    for k in ("triangles", "spread_count", "close_hist", "label_table", "open_close"):
        assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), k


PLANS = [
    # (tiny, small, large, huge) variants, tile caps
    ((0, 0, 0, 0), (1024,) * 4),
    ((V.TP_VAR_WAVE_TABLE, V.TP_VAR_GROUP_TABLE, V.TP_VAR_GROUP_TABLE, V.TP_VAR_SEARCH), (16,) * 4),
    ((V.TP_VAR_GROUP_TABLE, V.TP_VAR_SEARCH, V.TP_VAR_SEARCH, V.TP_VAR_WAVE_SEARCH), (256, 4096, 64, 65536)),
    ((V.TP_VAR_WAVE_SEARCH, V.TP_VAR_WAVE_SEARCH, V.TP_VAR_GROUP_TABLE, V.TP_VAR_SEARCH), (4096, 16, 16, 256)),
    ((V.TP_VAR_SEARCH, V.TP_VAR_GROUP_TABLE, V.TP_VAR_SEARCH, V.TP_VAR_SEARCH), (65536,) * 4),
]


@pytest.mark.parametrize("variants,caps", PLANS)
def test_plans_against_oracle(torch_cuda, mixed, variants, caps):
    torch = torch_cuda
    n, dev, ref = mixed
    stream = torch.cuda.current_stream().cuda_stream
    with tp.build_graph(n, *dev, stream=stream) as G:
        st = G.stats()
        assert st["class_tiles"][0] and st["class_tiles"][1] and st["class_tiles"][2]
        tp.tripoll_set_plan(G.handle, tp.make_plan(variants, caps), stream)
        assert tp.plan_dict(tp.tripoll_get_plan(G.handle)) == dict(variant=list(variants), tile_records=list(caps))
        st2 = G.stats()
        assert st2["probes"] == st["probes"] and st2["class_probes"] == st["class_probes"]
        say("plan", variants, caps, "tiles", st2["class_tiles"])
        got = tp.survey(G, stream=stream, outputs=OUT, n_labels=4, spread_lt=SPREAD)
        check(got, ref)
        assert got["probes"] == st["probes"]
        # and under the table-stress strategy (one cuckoo placement per key)
        check(tp.survey(G, stream=stream, outputs=OUT, n_labels=4, spread_lt=SPREAD,
                        strategy=tp.TP_STRAT_TABLE_STRESS), ref)


def test_tuner_choice_against_oracle(torch_cuda, mixed):
    torch = torch_cuda
    n, dev, ref = mixed
    stream = torch.cuda.current_stream().cuda_stream
    with tp.build_graph(n, *dev, stream=stream) as G:
        spec = tp.make_spec(outputs=OUT, n_labels=4, spread_lt=SPREAD)
        r = tp.tune_dict(tp.tripoll_tune(G.handle, spec, stream))
        say("tuned", r)
        assert r["trials"] >= 8
        assert tp.plan_dict(tp.tripoll_get_plan(G.handle)) == r["chosen"]
        for c, v in enumerate(r["chosen"]["variant"]):
            assert v in (0, 1, 2, 3, 4)
            assert r["chosen"]["tile_records"][c] in (256, 1024, 4096, 16384)
        check(tp.survey(G, stream=stream, outputs=OUT, n_labels=4, spread_lt=SPREAD), ref)


def test_huge_class_variants_closed_form(torch_cuda):
    """K_3400: targets of d+ > 3276 (the huge class) in pieces of Adj+(q) in
    LDS tables (the default), under both HBM search variants and small tile
    caps; C(n,3) triangles."""
    torch = torch_cuda
    n = 3400
    iu = np.triu_indices(n, 1)
    src, dst = [torch.from_numpy(x.astype(np.uint32)).cuda() for x in iu]
    stream = torch.cuda.current_stream().cuda_stream
    with tp.build_graph(n, src, dst, stream=stream) as G:
        assert G.stats()["class_tiles"][3] > 0
        for var, cap in ((V.TP_VAR_DEFAULT, 16384), (V.TP_VAR_GROUP_TABLE, 16), (V.TP_VAR_SEARCH, 1024),
                         (V.TP_VAR_WAVE_SEARCH, 1024), (V.TP_VAR_WAVE_SEARCH, 16)):
            tp.tripoll_set_plan(G.handle, tp.make_plan((0, 0, 0, var), (1024, 1024, 1024, cap)), stream)
            got = tp.survey(G, stream=stream, outputs=("count", "close_hist"))
            assert got["triangles"] == math.comb(n, 3)
            assert int(got["close_hist"][0]) == math.comb(n, 3)  # every time is 0


def test_set_plan_rejects_bad_plans(torch_cuda):
    torch = torch_cuda
    stream = torch.cuda.current_stream().cuda_stream
    src = torch.from_numpy(np.array([0, 1, 2], np.uint32)).cuda()
    dst = torch.from_numpy(np.array([1, 2, 0], np.uint32)).cuda()
    with tp.build_graph(3, src, dst, stream=stream) as G:
        bad = [((0, V.TP_VAR_WAVE_TABLE, 0, 0), (1024,) * 4),
               ((0, 0, 0, V.TP_VAR_WAVE_TABLE), (1024,) * 4),
               ((0, 0, 0, 9), (1024,) * 4),
               ((0, 0, 0, 0), (1000, 1024, 1024, 1024)),
               ((0, 0, 0, 0), (8, 1024, 1024, 1024)),
               ((0, 0, 0, 0), (1024, 1024, 1024, 1 << 17))]
        for variants, caps in bad:
            with pytest.raises(tp.TripollError) as e:
                tp.tripoll_set_plan(G.handle, tp.make_plan(variants, caps), stream)
            assert e.value.status == tp.TP_ERR_INVALID
        assert tp.survey(G, stream=stream)["triangles"] == 1
