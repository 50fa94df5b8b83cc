"""Independent brute-force survey used to pin the oracle (tests only).

Written from the definitions alone and sharing nothing with ``oracle.c``:
cleaning by a Python dict, triangles by checking vertex triples on a dense
adjacency matrix, closure bins by floating log2 (exact at these magnitudes),
label-multiset indices by listing the multisets in colex order.
"""
from __future__ import annotations

import math
from itertools import combinations_with_replacement

import numpy as np


def clean_dict(src, dst, ts):
    """{(lo, hi): earliest time} of the simple undirected graph."""
    best = {}
    for a, b, t in zip(src.tolist(), dst.tolist(), ts.tolist()):
        if a == b:
            continue
        k = (a, b) if a < b else (b, a)
        if k not in best or t < best[k]:
            best[k] = t
    return best


def ceil_log2_bin(d: int) -> int:
    """ceil(log2 d) as a histogram bin: d of 0 or 1 go to bin 0, cap at 31."""
    if d <= 1:
        return 0
    return min(31, math.ceil(math.log2(d)))


def colex_multisets(L: int):
    """All label multisets a<=b<=c over 0..L-1 in colex order, i.e. sorted by
    (c, b, a); maps each sorted triple to its position."""
    ms = sorted(combinations_with_replacement(range(L), 3), key=lambda x: (x[2], x[1], x[0]))
    return {m: i for i, m in enumerate(ms)}


def triangles(n: int, edges: dict):
    """All triangles (a<b<c) with their edge times, by vertex-triple checks
    on a dense adjacency matrix."""
    A = np.zeros((n, n), dtype=bool)
    T = np.zeros((n, n), dtype=np.int64)
    for (a, b), t in edges.items():
        A[a, b] = A[b, a] = True
        T[a, b] = T[b, a] = t
    out = []
    for a in range(n):
        for b in np.nonzero(A[a, a + 1:])[0] + a + 1:
            common = np.nonzero(A[a] & A[b])[0]
            for c in common[common > b]:
                out.append((a, int(b), int(c), int(T[a, b]), int(T[a, c]), int(T[b, c])))
    return out


def survey(n, src, dst, ts, vlab, n_labels=4, spread_lt=0, window=None, label_mask=None, max_edge_shift=0):
    edges = clean_dict(np.asarray(src), np.asarray(dst), np.asarray(ts))
    tris = triangles(n, edges)
    idx_of = colex_multisets(n_labels)
    deg_idx = colex_multisets(32)
    degree = [0] * n
    for a, b in edges:
        degree[a] += 1
        degree[b] += 1
    res = dict(triangles=0, spread_count=0, close_hist=np.zeros(32, np.uint64),
               label_table=np.zeros(len(idx_of), np.uint64), open_close=np.zeros((32, 32), np.uint64),
               max_edge=np.zeros(1024, np.uint64), degree_table=np.zeros(len(deg_idx), np.uint64),
               max_edge_exact={}, m=len(edges), tris=tris)
    for a, b, c, tab, tac, tbc in tris:
        times = sorted((tab, tac, tbc))
        if window is not None and not all(window[0] <= x <= window[1] for x in times):
            continue
        labs = tuple(sorted((int(vlab[a]), int(vlab[b]), int(vlab[c]))))
        idx = idx_of[labs]
        if label_mask is not None and idx not in label_mask:
            continue
        close = times[2] - times[0]
        opn = times[1] - times[0]
        res["triangles"] += 1
        res["close_hist"][ceil_log2_bin(close)] += 1
        res["label_table"][idx] += 1
        res["open_close"][ceil_log2_bin(opn), ceil_log2_bin(close)] += 1
        if close < spread_lt:
            res["spread_count"] += 1
        # Algorithm 3: pairwise distinct vertex labels, largest edge time
        if len({int(vlab[a]), int(vlab[b]), int(vlab[c])}) == 3:
            res["max_edge"][min(1023, times[2] // 2 ** max_edge_shift)] += 1
            # and its exact counting set: largest time -> triangles
            res["max_edge_exact"][times[2]] = res["max_edge_exact"].get(times[2], 0) + 1
        # degree metadata: sorted triple of ceil(log2 d)
        dl = tuple(sorted(ceil_log2_bin(degree[x]) for x in (a, b, c)))
        res["degree_table"][deg_idx[dl]] += 1
    return res


# representatives of the seven directed triangle types, as arc lists on
# vertices 0, 1, 2 (triad census names)
_DIRECTED_REPS = {
    0: [(0, 1), (0, 2), (1, 2)],                          # 030T
    1: [(0, 1), (1, 2), (2, 0)],                          # 030C
    2: [(0, 1), (0, 2), (1, 2), (2, 1)],                  # 120D
    3: [(1, 0), (2, 0), (1, 2), (2, 1)],                  # 120U
    4: [(0, 1), (2, 0), (1, 2), (2, 1)],                  # 120C
    5: [(0, 1), (1, 0), (0, 2), (2, 0), (1, 2)],          # 210
    6: [(0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1)],  # 300
}


def _canon_arcs(arcs):
    """Smallest arc set over the six relabellings of 0, 1, 2."""
    from itertools import permutations
    return min(tuple(sorted((pi[a], pi[b]) for a, b in arcs)) for pi in permutations(range(3)))


_DIRECTED_CANON = {_canon_arcs(a): t for t, a in _DIRECTED_REPS.items()}


def directed_census(n, src, dst):
    """Census of directed triangle types of a directed multigraph (self-loops
    and repeated arcs ignored), by matching each triangle's arc set to the
    representatives up to relabelling."""
    arcs = {(int(a), int(b)) for a, b in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()) if a != b}
    und = {}
    for a, b in arcs:
        und.setdefault((min(a, b), max(a, b)), set()).add((a, b))
    out = np.zeros(7, np.uint64)
    for a, b, c, *_ in triangles(n, {k: 0 for k in und}):
        idx = {a: 0, b: 1, c: 2}
        sub = [(idx[x], idx[y]) for pair in ((a, b), (a, c), (b, c)) for x, y in und[pair]]
        out[_DIRECTED_CANON[_canon_arcs(sub)]] += 1
    return out
