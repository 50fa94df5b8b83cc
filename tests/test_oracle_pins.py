"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it cannot agree with by
construction: hand-worked values, closed forms, an independent brute force,
exact linear algebra (trace(A^3)/6), or invariances of the definition.
"""
import json
import math
import os
from itertools import combinations

import numpy as np
import pytest

import oracle
import synth
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL_OUT = ("count", "close_hist", "label_table", "spread_count", "open_close", "max_edge", "degree_table")


def run(n, edges, labels=None, **kw):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    src, dst, ts = (e[:, i].astype(np.uint32) for i in range(3))
    vlab = np.zeros(n, np.uint8) if labels is None else np.asarray(labels, np.uint8)
    kw.setdefault("outputs", ALL_OUT)
    return oracle.survey(n, src, dst, ts, vlab, **kw)


def complete(n, t=lambda u, v: 0):
    return [(u, v, t(u, v)) for u, v in combinations(range(n), 2)]


# -------------------------------------------------------------- callback math

def test_bin_table():
    # ceil(log2 D) worked by hand; D = 0 and D = 1 share bin 0; cap at 31
    table = {0: 0, 1: 0, 2: 1, 3: 2, 4: 2, 5: 3, 8: 3, 9: 4, 1000: 10, 1024: 10, 1025: 11,
             65535: 16, 65536: 16, 65537: 17, 2 ** 31: 31, 2 ** 31 + 1: 31, 2 ** 32 - 1: 31}
    for d, b in table.items():
        assert oracle.bin_of(d) == b, d
    for k in range(1, 31):
        assert oracle.bin_of(2 ** k) == k
        assert oracle.bin_of(2 ** k + 1) == k + 1
        assert oracle.bin_of(2 ** k - 1) == (k if k > 1 else 0)


def test_msidx_small_values_and_bijection():
    # colex order of multisets: 000,001,011,111,002,012,112,022,122,222,003,...
    first = [(0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1), (0, 0, 2), (0, 1, 2), (1, 1, 2),
             (0, 2, 2), (1, 2, 2), (2, 2, 2), (0, 0, 3)]
    for i, m in enumerate(first):
        assert oracle.msidx(*m) == i
        assert oracle.msidx(*reversed(m)) == i
    for L in (1, 2, 4, 8, 16):
        ref = brute.colex_multisets(L)
        got = {m: oracle.msidx(*m) for m in ref}
        assert got == ref
        assert sorted(got.values()) == list(range(oracle.table_size(L)))
    assert oracle.table_size(4) == 20 and oracle.table_size(8) == 120


# -------------------------------------------------------------- hand-worked

def test_hand_worked_fixture():
    fx = json.load(open(os.path.join(GOLDEN, "tiny_hand.json")))
    n, labels, edges, ex = fx["n"], fx["labels"], fx["edges"], fx["expect"]
    r = run(n, edges, labels, n_labels=fx["n_labels"], spread_lt=ex["spread_lt"], records=True)
    assert r["m"] == fx["unique_edges"]
    assert r["triangles"] == ex["triangles"]
    hist = np.zeros(32, np.uint64)
    for b, c in ex["close_hist"].items():
        hist[int(b)] = c
    assert (r["close_hist"] == hist).all()
    tab = np.zeros(20, np.uint64)
    for i, c in ex["label_table"].items():
        tab[int(i)] = c
    assert (r["label_table"] == tab).all()
    assert r["spread_count"] == ex["spread_count"]
    oc = np.zeros((32, 32), np.uint64)
    for k, c in ex["open_close"].items():
        o, cl = map(int, k.split(","))
        oc[o, cl] = c
    assert (r["open_close"] == oc).all()
    got = sorted(map(tuple, np.stack([r["records"][f] for f in "abc"], 1).tolist()))
    assert got == [tuple(x) for x in ex["triangles_sorted"]]
    w = run(n, edges, labels, n_labels=4, window=ex["window"])
    assert w["triangles"] == ex["window_triangles"]
    lm = run(n, edges, labels, n_labels=4, label_mask=ex["label_mask"])
    assert lm["triangles"] == ex["label_mask_triangles"]


# -------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [3, 4, 5, 10, 33, 64])
def test_complete_graph(n):
    r = run(n, complete(n))
    assert r["triangles"] == math.comb(n, 3)
    assert r["wedges"] == math.comb(n, 3)  # every wedge of K_n closes
    assert r["close_hist"][0] == math.comb(n, 3)


@pytest.mark.parametrize("k", [1, 5, 16, 30])
def test_complete_graph_time_bins(k):
    # ts(u,v) = 7 + 2^k if 0 in {u,v} else 7: triangles through 0 have spread 2^k
    n = 12
    r = run(n, complete(n, lambda u, v: 7 + (2 ** k if 0 in (u, v) else 0)), spread_lt=2 ** k)
    hist = np.zeros(32, np.uint64)
    hist[k] += math.comb(n - 1, 2)
    hist[0] += math.comb(n - 1, 3)
    assert (r["close_hist"] == hist).all()
    assert r["spread_count"] == math.comb(n - 1, 3)  # spread 2^k is not < 2^k
    # a triangle through 0 has sorted times (7, 7+2^k, 7+2^k): open 2^k, close 2^k
    assert r["open_close"][k, k] == math.comb(n - 1, 2)


def test_complete_graph_label_classes():
    sizes = [5, 3, 0, 4]
    labels = sum(([c] * s for c, s in enumerate(sizes)), [])
    n = len(labels)
    r = run(n, complete(n), labels, n_labels=4)
    exp = np.zeros(20, np.uint64)
    for a in range(4):
        for b in range(a, 4):
            for c in range(b, 4):
                if a == b == c:
                    cnt = math.comb(sizes[a], 3)
                elif a == b:
                    cnt = math.comb(sizes[a], 2) * sizes[c]
                elif b == c:
                    cnt = sizes[a] * math.comb(sizes[b], 2)
                else:
                    cnt = sizes[a] * sizes[b] * sizes[c]
                exp[brute.colex_multisets(4)[(a, b, c)]] = cnt
    assert (r["label_table"] == exp).all()
    assert r["label_table"].sum() == math.comb(n, 3)


# -------------------------------------------------------------- Algorithm 3 and degree triples


@pytest.mark.parametrize("n,shift", [(8, 0), (16, 0), (16, 2), (40, 0), (40, 3)])
def test_max_edge_complete_graph_closed_form(n, shift):
    # K_n with ts(u,v) = max(u,v): the largest edge time of triangle a<b<c is c,
    # and vertex c closes C(c,2) triangles; distinct labels (v mod 16) hold for
    # all triangles when n <= 16 and for those with distinct residues otherwise
    labels = [v % 16 for v in range(n)]
    r = run(n, complete(n, lambda u, v: max(u, v)), labels, n_labels=16, max_edge_shift=shift)
    exp = np.zeros(1024, np.uint64)
    for c in range(n):
        for a, b in combinations(range(c), 2):
            if len({labels[a], labels[b], labels[c]}) == 3:
                exp[c >> shift] += 1
    if n <= 16:
        assert exp.sum() == math.comb(n, 3)
        for c in range(n):
            assert int(exp[c]) == math.comb(c, 2) or shift
    assert (r["max_edge"] == exp).all()


def test_max_edge_label_classes_and_saturation():
    # three label classes: every distinct-label triangle takes one vertex of
    # each class, n_a*n_b*n_c of them; two classes give none
    sizes = [4, 3, 5]
    labels = sum(([c] * s for c, s in enumerate(sizes)), [])
    n = len(labels)
    r = run(n, complete(n, lambda u, v: 5000 + u + v), labels, n_labels=4, max_edge_shift=0)
    assert r["max_edge"].sum() == 4 * 3 * 5
    assert r["max_edge"][1023] == 4 * 3 * 5  # every time >= 1023 lands in the last bin
    r2 = run(n, complete(n), [0 if x < 2 else 1 for x in labels], n_labels=4)
    assert r2["max_edge"].sum() == 0
    # the distinct-label triangles are exactly the label-table cells a<b<c
    idx = brute.colex_multisets(4)
    assert r["max_edge"].sum() == sum(int(r["label_table"][idx[(a, b, c)]])
                                      for a, b, c in combinations(range(4), 3))


def _exact_dict(vals, cnts):
    assert (np.diff(vals.astype(np.int64)) > 0).all()  # ascending, each value once
    return dict(zip(vals.tolist(), cnts.tolist()))


@pytest.mark.parametrize("n", [3, 8, 16])
def test_max_edge_exact_complete_graph_closed_form(n):
    # K_n, ts(u,v) = max(u,v), labels = ids: every triangle a<b<c has largest
    # time c, and c closes C(c,2) of them, so the counting set is {c: C(c,2)}
    e = np.array(complete(n, lambda u, v: max(u, v)), np.int64).reshape(-1, 3)
    vals, cnts = oracle.max_edge_counts(n, e[:, 0].astype(np.uint32), e[:, 1].astype(np.uint32),
                                        e[:, 2].astype(np.uint32), np.arange(n, dtype=np.uint8), n_labels=16)
    assert _exact_dict(vals, cnts) == {c: math.comb(c, 2) for c in range(2, n)}


def test_max_edge_exact_degenerate():
    # no distinct-label triangle (two label classes), no triangle, no edge
    n = 10
    e = np.array(complete(n, lambda u, v: u * v), np.int64).reshape(-1, 3)
    s, d, t = (e[:, i].astype(np.uint32) for i in range(3))
    vals, cnts = oracle.max_edge_counts(n, s, d, t, (np.arange(n) % 2).astype(np.uint8))
    assert len(vals) == 0 and len(cnts) == 0
    star = np.arange(1, n, dtype=np.uint32)
    vals, _ = oracle.max_edge_counts(n, np.zeros(n - 1, np.uint32), star, star, np.arange(n, dtype=np.uint8),
                                     n_labels=16)
    assert len(vals) == 0
    vals, _ = oracle.max_edge_counts(n, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                                     np.zeros(n, np.uint8))
    assert len(vals) == 0


@pytest.mark.parametrize("seed,n,M,L", [(11, 40, 400, 3), (12, 90, 1800, 4), (13, 150, 3000, 8),
                                        (14, 60, 1500, 16)])
def test_max_edge_exact_against_brute_force(seed, n, M, L):
    # the exact counting set against the brute force, with and without the
    # filters; summed into bins it is the binned output of Algorithm 3
    rng = np.random.default_rng(seed)
    src, dst, ts, vlab = _random_graph(rng, n, M, tbits=int(rng.integers(4, 33)), L=L)
    b = brute.survey(n, src, dst, ts, vlab, n_labels=L)
    vals, cnts = oracle.max_edge_counts(n, src, dst, ts, vlab, n_labels=L)
    assert _exact_dict(vals, cnts) == b["max_edge_exact"]
    for shift in (0, 5, 20):
        r = oracle.survey(n, src, dst, ts, vlab, outputs=("max_edge",), n_labels=L, max_edge_shift=shift)
        binned = np.zeros(1024, np.uint64)
        np.add.at(binned, np.minimum(vals.astype(np.int64) >> shift, 1023), cnts)
        assert (binned == r["max_edge"]).all()
    lo, hi = np.quantile(ts.astype(np.float64), [0.2, 0.9]).astype(np.int64)
    mask = set(range(0, brute.colex_multisets(L).__len__(), 3))
    b = brute.survey(n, src, dst, ts, vlab, n_labels=L, window=(lo, hi), label_mask=mask)
    vals, cnts = oracle.max_edge_counts(n, src, dst, ts, vlab, n_labels=L, window=(lo, hi), label_mask=mask)
    assert _exact_dict(vals, cnts) == b["max_edge_exact"]


def test_max_edge_shift_range():
    with pytest.raises(ValueError):
        run(4, complete(4), outputs=("count", "max_edge"), max_edge_shift=32)


@pytest.mark.parametrize("n", [3, 4, 5, 9, 17, 33])
def test_degree_table_complete_graph(n):
    # every vertex of K_n has degree n-1
    b = oracle.bin_of(n - 1)
    r = run(n, complete(n))
    exp = np.zeros(oracle.DEGREE_MAX, np.uint64)
    exp[brute.colex_multisets(32)[(b, b, b)]] = math.comb(n, 3)
    assert (r["degree_table"] == exp).all()


@pytest.mark.parametrize("k", [2, 3, 5, 9, 100])
def test_degree_table_friendship_and_wheel(k):
    idx = brute.colex_multisets(32)
    # friendship graph F_k: centre of degree 2k, blades of degree 2
    fr = []
    for i in range(k):
        a, c = 1 + 2 * i, 2 + 2 * i
        fr += [(0, a, 0), (0, c, 0), (a, c, 0)]
    r = run(2 * k + 1, fr)
    exp = np.zeros(oracle.DEGREE_MAX, np.uint64)
    exp[idx[tuple(sorted((1, 1, math.ceil(math.log2(2 * k)))))]] = k
    assert (r["degree_table"] == exp).all()
    # wheel of k >= 4 spokes: hub degree k, rim degree 3 (ceil(log2 3) = 2)
    if k >= 4:
        wheel = [(0, i, 0) for i in range(1, k + 1)] + [(i, i % k + 1, 0) for i in range(1, k + 1)]
        r = run(k + 1, wheel)
        exp = np.zeros(oracle.DEGREE_MAX, np.uint64)
        exp[idx[(2, 2, math.ceil(math.log2(k)))]] = k
        assert (r["degree_table"] == exp).all()


def test_zero_triangle_families():
    star = [(0, i, i) for i in range(1, 50)]
    assert run(50, star)["triangles"] == 0
    assert run(50, star)["wedges"] == 0  # the hub is last in degree order
    kab = [(u, 10 + v, 1) for u in range(10) for v in range(7)]
    assert run(17, kab)["triangles"] == 0
    # Petersen graph: girth 5
    outer = [(i, (i + 1) % 5, 0) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5, 0) for i in range(5)]
    spokes = [(i, 5 + i, 0) for i in range(5)]
    assert run(10, outer + inner + spokes)["triangles"] == 0


@pytest.mark.parametrize("k", [4, 5, 9, 100])
def test_wheel_and_friendship(k):
    wheel = [(0, i, 0) for i in range(1, k + 1)] + [(i, i % k + 1, 0) for i in range(1, k + 1)]
    assert run(k + 1, wheel)["triangles"] == k
    fr = []
    for i in range(k):
        a, b = 1 + 2 * i, 2 + 2 * i
        fr += [(0, a, 0), (0, b, 0), (a, b, 0)]
    assert run(2 * k + 1, fr)["triangles"] == k


def test_platonic_solids():
    # octahedron K_{2,2,2}: 8 triangular faces, no other triangles
    octa = [(u, v, 0) for u, v in combinations(range(6), 2) if u // 2 != v // 2]
    assert run(6, octa)["triangles"] == 8
    # icosahedron: 20 faces; vertices 0 (top), 1..5 upper ring, 6..10 lower ring, 11 bottom
    e = [(0, i, 0) for i in range(1, 6)] + [(11, i, 0) for i in range(6, 11)]
    e += [(i, i % 5 + 1, 0) for i in range(1, 6)] + [(i, (i - 5) % 5 + 6, 0) for i in range(6, 11)]
    e += [(i, i + 5, 0) for i in range(1, 6)] + [(i, i % 5 + 6, 0) for i in range(1, 6)]
    assert len({tuple(sorted(x[:2])) for x in e}) == 30
    assert run(12, e)["triangles"] == 20


def test_disjoint_triangles():
    e = []
    for i in range(40):
        a = 3 * i
        e += [(a, a + 1, i), (a + 1, a + 2, i), (a, a + 2, i)]
    r = run(120, e)
    assert r["triangles"] == 40 and r["close_hist"][0] == 40


# -------------------------------------------------------------- filters

def test_spread_boundary():
    e = [(0, 1, 0), (1, 2, 0), (0, 2, 2 ** 16 - 1), (3, 4, 0), (4, 5, 0), (3, 5, 2 ** 16)]
    r = run(6, e, spread_lt=2 ** 16)
    assert r["triangles"] == 2 and r["spread_count"] == 1
    assert run(6, e, spread_lt=2 ** 64 - 1)["spread_count"] == 2
    assert run(6, e, spread_lt=0)["spread_count"] == 0


def test_window_filter():
    e = [(0, 1, 10), (1, 2, 20), (0, 2, 30), (3, 4, 0), (4, 5, 2 ** 32 - 1), (3, 5, 5)]
    assert run(6, e, window=(0, 2 ** 32 - 1))["triangles"] == 2
    assert run(6, e, window=(10, 30))["triangles"] == 1
    assert run(6, e, window=(11, 30))["triangles"] == 0
    assert run(6, e, window=(10, 29))["triangles"] == 0
    assert run(6, e, window=(40, 50))["triangles"] == 0


# -------------------------------------------------------------- brute force

def _random_graph(rng, n, M, tbits=12, L=4):
    src = rng.integers(0, n, M).astype(np.uint32)
    dst = rng.integers(0, n, M).astype(np.uint32)
    ts = rng.integers(0, 2 ** tbits, M).astype(np.uint32)
    vlab = rng.integers(0, L, n).astype(np.uint8)
    # force duplicates, reversed copies and self-loops
    k = M // 8
    src = np.concatenate([src, dst[:k], src[:k], src[:k]])
    dst = np.concatenate([dst, src[:k], dst[:k], src[:k]])
    ts = np.concatenate([ts, ts[:k] + 1, ts[:k] // 2, ts[:k]])
    return src, dst, ts, vlab


@pytest.mark.parametrize("seed,n,M,L", [(1, 30, 200, 2), (2, 60, 700, 4), (3, 120, 2500, 8),
                                        (4, 200, 1500, 16), (5, 50, 1225, 3)])
def test_against_brute_force(seed, n, M, L):
    rng = np.random.default_rng(seed)
    src, dst, ts, vlab = _random_graph(rng, n, M, tbits=rng.integers(1, 33), L=L)
    b = brute.survey(n, src, dst, ts, vlab, n_labels=L, spread_lt=2 ** 8)
    r = oracle.survey(n, src, dst, ts, vlab, outputs=ALL_OUT, n_labels=L, spread_lt=2 ** 8,
                      records=True)
    assert r["m"] == b["m"]
    assert r["triangles"] == b["triangles"]
    assert (r["close_hist"] == b["close_hist"]).all()
    assert (r["label_table"] == b["label_table"]).all()
    assert (r["open_close"] == b["open_close"]).all()
    assert (r["max_edge"] == b["max_edge"]).all()
    assert (r["degree_table"] == b["degree_table"]).all()
    assert r["spread_count"] == b["spread_count"]
    # exactly once, with the same six metadata items
    rec = r["records"]
    got = sorted(zip(*(rec[f].tolist() for f in ("a", "b", "c", "t_ab", "t_ac", "t_bc"))))
    assert len(set(g[:3] for g in got)) == len(got)
    assert got == sorted(b["tris"])
    for x in rec:
        assert (x["l_a"], x["l_b"], x["l_c"]) == (vlab[x["a"]], vlab[x["b"]], vlab[x["c"]])


def test_against_brute_force_filters():
    rng = np.random.default_rng(9)
    n, L = 80, 4
    src, dst, ts, vlab = _random_graph(rng, n, 1500, tbits=10, L=L)
    for window in [(100, 900), (0, 1023), (512, 512)]:
        b = brute.survey(n, src, dst, ts, vlab, n_labels=L, window=window)
        r = oracle.survey(n, src, dst, ts, vlab, outputs=ALL_OUT, n_labels=L, window=window)
        assert r["triangles"] == b["triangles"]
        assert (r["close_hist"] == b["close_hist"]).all()
    mask = {0, 5, 7, 19}
    b = brute.survey(n, src, dst, ts, vlab, n_labels=L, label_mask=mask)
    r = oracle.survey(n, src, dst, ts, vlab, outputs=ALL_OUT, n_labels=L, label_mask=mask)
    assert r["triangles"] == b["triangles"]
    assert (r["label_table"] == b["label_table"]).all()


def test_rmat_small_against_brute_force():
    w = synth.workload(1, scale=8)
    g = synth.generate(w.graph)
    b = brute.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], n_labels=4)
    r = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], outputs=ALL_OUT, n_labels=4)
    assert r["triangles"] == b["triangles"] > 0
    assert (r["close_hist"] == b["close_hist"]).all()
    assert (r["label_table"] == b["label_table"]).all()


# -------------------------------------------------------------- linear algebra

def _adj(n, u, v):
    A = np.zeros((n, n))
    A[u, v] = 1
    A[v, u] = 1
    return A


def test_trace_a3_on_scale12_workload():
    # trace(A^3)/6 in float64 is exact here (all partial sums < 2^53)
    w = synth.workload(1)
    g = synth.generate(w.graph)
    u, v, t = oracle.clean(g["n"], g["src"], g["dst"], g["ts"])
    A = _adj(g["n"], u, v)
    tri = int(round(np.trace(A @ A @ A) / 6))
    r = oracle.survey_clean(g["n"], u, v, t, g["vlab"], outputs=("count",))
    assert r["triangles"] == tri
    # wedges of the DODGr: sum over v of C(d+(v), 2) >= T
    assert r["wedges"] >= tri


def test_sparse_hadamard_scale14():
    import scipy.sparse as sp
    w = synth.workload(1, scale=14)
    g = synth.generate(w.graph)
    u, v, t = oracle.clean(g["n"], g["src"], g["dst"], g["ts"])
    n = g["n"]
    A = sp.coo_matrix((np.ones(len(u)), (u, v)), shape=(n, n)).tocsr()
    A = (A + A.T).tocsr()
    tri = int(round(A.multiply(A @ A).sum() / 6))
    r = oracle.survey_clean(n, u, v, t, g["vlab"], outputs=("count",))
    assert r["triangles"] == tri


def test_cleaning_matches_dict():
    rng = np.random.default_rng(4)
    src, dst, ts, vlab = _random_graph(rng, 300, 5000, tbits=20)
    u, v, t = oracle.clean(300, src, dst, ts)
    d = brute.clean_dict(src, dst, ts)
    assert sorted(zip(u.tolist(), v.tolist(), t.tolist())) == sorted((a, b, c) for (a, b), c in d.items())
    with pytest.raises(ValueError):
        oracle.clean(10, np.array([1, 10], np.uint32), np.array([2, 3], np.uint32), None)


# -------------------------------------------------------------- invariances

def _results_equal(a, b, keys=("triangles", "spread_count", "close_hist", "label_table", "open_close")):
    for k in keys:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_invariant_to_duplicates_loops_and_order():
    w = synth.workload(1, scale=10)
    g = synth.generate(w.graph)
    kw = dict(outputs=ALL_OUT, n_labels=4, spread_lt=2 ** 18)
    base = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], **kw)
    rng = np.random.default_rng(0)
    M = len(g["src"])
    pick = rng.integers(0, M, M // 3)
    src = np.concatenate([g["src"], g["dst"][pick], g["src"][pick], np.arange(50, dtype=np.uint32)])
    dst = np.concatenate([g["dst"], g["src"][pick], g["dst"][pick], np.arange(50, dtype=np.uint32)])
    ts = np.concatenate([g["ts"], g["ts"][pick] + 5, g["ts"][pick] + 1, np.zeros(50, np.uint32)])
    perm = rng.permutation(len(src))
    r = oracle.survey(g["n"], src[perm], dst[perm], ts[perm], g["vlab"], **kw)
    _results_equal(base, r)


def test_invariant_to_vertex_relabelling():
    w = synth.workload(1, scale=10)
    g = synth.generate(w.graph)
    kw = dict(outputs=ALL_OUT, n_labels=4, spread_lt=2 ** 18)
    base = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], **kw)
    pi = np.random.default_rng(3).permutation(g["n"]).astype(np.uint32)
    vlab = np.empty_like(g["vlab"])
    vlab[pi] = g["vlab"]
    r = oracle.survey(g["n"], pi[g["src"]], pi[g["dst"]], g["ts"], vlab, **kw)
    _results_equal(base, r)
    assert r["triangles"] > 0


def test_sums_equal_triangles():
    w = synth.workload(1)
    g = synth.generate(w.graph)
    r = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], outputs=ALL_OUT, n_labels=4)
    assert r["close_hist"].sum() == r["label_table"].sum() == r["open_close"].sum() == r["triangles"]
    assert r["degree_table"].sum() == r["triangles"]
    idx = brute.colex_multisets(4)
    distinct = sum(int(r["label_table"][idx[(a, b, c)]]) for a, b, c in combinations(range(4), 3))
    assert r["max_edge"].sum() == distinct > 0


def test_label_out_of_range_rejected():
    with pytest.raises(ValueError):
        run(3, complete(3), [0, 1, 5], n_labels=4)


# -------------------------------------------------------------- local participation

def part(n, edges, labels=None, **kw):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    src, dst, ts = (e[:, i].astype(np.uint32) for i in range(3))
    vlab = np.zeros(n, np.uint8) if labels is None else np.asarray(labels, np.uint8)
    vc, (u, v, t, ec) = oracle.participation(n, src, dst, ts, vlab, **kw)
    return vc, {(int(a), int(b)): int(c) for a, b, c in zip(u, v, ec)}


@pytest.mark.parametrize("n", [3, 4, 7, 20])
def test_participation_complete_graph(n):
    vc, ec = part(n, complete(n))
    assert (vc == math.comb(n - 1, 2)).all()
    assert len(ec) == math.comb(n, 2) and set(ec.values()) == {n - 2}


@pytest.mark.parametrize("k", [4, 5, 12])
def test_participation_wheel_and_friendship(k):
    wheel = [(0, i, 0) for i in range(1, k + 1)] + [(i, i % k + 1, 0) for i in range(1, k + 1)]
    vc, ec = part(k + 1, wheel)
    assert vc[0] == k and (vc[1:] == 2).all()
    for (a, b), c in ec.items():
        assert c == (2 if a == 0 else 1)
    fr = []
    for i in range(k):
        a, b = 1 + 2 * i, 2 + 2 * i
        fr += [(0, a, 0), (0, b, 0), (a, b, 0)]
    vc, ec = part(2 * k + 1, fr)
    assert vc[0] == k and (vc[1:] == 1).all() and set(ec.values()) == {1}


@pytest.mark.parametrize("seed", range(4))
def test_participation_against_brute_force(seed):
    rng = np.random.default_rng(40 + seed)
    n, L = int(rng.integers(30, 150)), 4
    src, dst, ts, vlab = _random_graph(rng, n, int(rng.integers(n, 12 * n)), tbits=12, L=L)
    window = None if seed % 2 == 0 else (500, 3500)
    mask = None if seed < 2 else [0, 3, 7, 11, 19]
    b = brute.survey(n, src, dst, ts, vlab, n_labels=L)
    idx_of = brute.colex_multisets(L)
    want_v = np.zeros(n, np.uint64)
    want_e = {}
    kept = 0
    for a, bb, c, tab, tac, tbc in b["tris"]:
        if window is not None and not all(window[0] <= x <= window[1] for x in (tab, tac, tbc)):
            continue
        if mask is not None and idx_of[tuple(sorted((int(vlab[a]), int(vlab[bb]), int(vlab[c]))))] not in mask:
            continue
        kept += 1
        for x in (a, bb, c):
            want_v[x] += 1
        for e in ((a, bb), (a, c), (bb, c)):
            want_e[e] = want_e.get(e, 0) + 1
    vc, (u, v, t, ec) = oracle.participation(n, src, dst, ts, vlab, n_labels=L, window=window, label_mask=mask)
    assert np.array_equal(vc, want_v)
    got_e = {(int(a), int(bb)): int(c) for a, bb, c in zip(u, v, ec) if c}
    assert got_e == want_e
    # each triangle at v holds two of v's edges
    half = np.zeros(n, np.uint64)
    np.add.at(half, u, ec)
    np.add.at(half, v, ec)
    assert np.array_equal(half, 2 * vc)
    assert vc.sum() == ec.sum() == 3 * kept


def test_participation_sums_on_workload1():
    w = synth.workload(1)
    g = synth.generate(w.graph)
    r = oracle.survey(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], outputs=("count",), n_labels=4)
    vc, (u, v, t, ec) = oracle.participation(g["n"], g["src"], g["dst"], g["ts"], g["vlab"], n_labels=4)
    assert vc.sum() == ec.sum() == 3 * r["triangles"]


# -------------------------------------------------------------- directed census

def dsurvey(n, arcs):
    a = np.asarray(arcs, dtype=np.int64).reshape(-1, 2)
    src, dst = a[:, 0].astype(np.uint32), a[:, 1].astype(np.uint32)
    return oracle.survey(n, src, dst, np.zeros(len(a), np.uint32), np.zeros(n, np.uint8),
                         outputs=("count", "directed"))


def test_directed_types_of_single_triangles():
    for t, arcs in brute._DIRECTED_REPS.items():
        r = dsurvey(3, arcs)
        exp = np.zeros(7, np.uint64)
        exp[t] = 1
        assert (r["directed"] == exp).all(), (oracle.DIRECTED_TYPES[t], r["directed"])
    # a repeated arc or a reversed copy changes the pair's directions
    assert dsurvey(3, [(0, 1), (1, 2), (2, 0), (0, 1)])["directed"][1] == 1
    assert dsurvey(3, [(0, 1), (1, 2), (2, 0), (1, 0)])["directed"][4] == 1


@pytest.mark.parametrize("n,seed", [(5, 1), (12, 2), (30, 3)])
def test_directed_tournament_closed_form(n, seed):
    # a random tournament: C(n,3) triangles, of which sum_v C(out(v), 2) are
    # transitive (one per vertex that sends both of its arcs) and the rest cyclic
    rng = np.random.default_rng(seed)
    arcs = [(u, v) if rng.random() < 0.5 else (v, u) for u, v in combinations(range(n), 2)]
    out = np.bincount([a for a, _ in arcs], minlength=n)
    r = dsurvey(n, arcs)
    trans = sum(math.comb(int(k), 2) for k in out)
    assert r["directed"][0] == trans and r["directed"][1] == math.comb(n, 3) - trans
    assert r["directed"][2:].sum() == 0
    # every pair in both directions: all mutual
    both = arcs + [(b, a) for a, b in arcs]
    assert dsurvey(n, both)["directed"][6] == math.comb(n, 3)


@pytest.mark.parametrize("seed", range(4))
def test_directed_against_brute_force(seed):
    rng = np.random.default_rng(60 + seed)
    n = int(rng.integers(10, 70))
    M = int(rng.integers(n, 10 * n))
    src = rng.integers(0, n, M).astype(np.uint32)
    dst = rng.integers(0, n, M).astype(np.uint32)
    r = oracle.survey(n, src, dst, np.zeros(M, np.uint32), np.zeros(n, np.uint8), outputs=("count", "directed"))
    assert (r["directed"] == brute.directed_census(n, src, dst)).all()
    assert r["directed"].sum() == r["triangles"]
