"""CPU oracle of the metadata triangle survey -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (``paper_2107_12330_amd``) never
touches it, and the two share no code.  The arithmetic lives in ``oracle.c``
(plain C, OpenMP over pivots); this wrapper only marshals arguments.

Survey outputs are selected by name:
  "count"         number of triangles (Algorithm 2)
  "close_hist"    32 bins of ceil(log2(max t - min t)) (Algorithm 4, close)
  "label_table"   counts per sorted vertex-label multiset (colex index)
  "spread_count"  triangles with max t - min t < spread_lt
  "open_close"    32 x 32 joint (open, close) bins (Algorithm 4)
  "max_edge"      Algorithm 3: over triangles with pairwise distinct vertex
                  labels, counts of the largest edge time t3 in 1024 bins
                  t3 >> max_edge_shift (the last bin takes the rest);
                  max_edge_counts() gives its exact counting set
  "degree_table"  counts per sorted triple of ceil(log2 d(v)) over the three
                  vertices (the degree metadata of the evaluation), indexed
                  like the label table, 5984 entries (values 0..31)
  "directed"      census of directed triangle types (030T, 030C, 120D, 120U,
                  120C, 210, 300) from the directions of the raw edges
Filters: window=(t_lo, t_hi) keeps triangles whose three times lie in the
closed range; label_mask=set of multiset indices keeps only those.

participation() gives the local counts: triangles at each vertex and at each
edge of the cleaned graph, under the same filters.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OUT_BITS = {"count": 1, "close_hist": 2, "label_table": 4, "spread_count": 8, "open_close": 16,
            "max_edge": 32, "degree_table": 64, "directed": 128}
DIRECTED_TYPES = ("030T", "030C", "120D", "120U", "120C", "210", "300")
TABLE_MAX = 816
MAX_EDGE_BINS = 1024
DEGREE_MAX = 5984  # C(34, 3): multisets of three values in 0..31


class _Spec(ctypes.Structure):
    _fields_ = [("outputs", ctypes.c_uint32), ("filters", ctypes.c_uint32),
                ("n_labels", ctypes.c_uint32), ("max_edge_shift", ctypes.c_uint32),
                ("spread_lt", ctypes.c_uint64), ("t_lo", ctypes.c_uint64), ("t_hi", ctypes.c_uint64),
                ("label_mask", ctypes.c_uint64 * ((TABLE_MAX + 63) // 64))]


class _Result(ctypes.Structure):
    _fields_ = [("triangles", ctypes.c_uint64), ("spread_count", ctypes.c_uint64),
                ("wedges", ctypes.c_uint64), ("close_hist", ctypes.c_uint64 * 32),
                ("label_table", ctypes.c_uint64 * TABLE_MAX),
                ("open_close", ctypes.c_uint64 * 1024),
                ("max_edge", ctypes.c_uint64 * MAX_EDGE_BINS),
                ("degree_table", ctypes.c_uint64 * DEGREE_MAX),
                ("directed", ctypes.c_uint64 * 7)]


TRI_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("c", "<u4"),
                      ("t_ab", "<u4"), ("t_ac", "<u4"), ("t_bc", "<u4"),
                      ("l_a", "u1"), ("l_b", "u1"), ("l_c", "u1"), ("pad", "u1")])

_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", _LIB + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    p = ctypes.c_void_p
    lib.oracle_bin.restype = ctypes.c_uint32
    lib.oracle_bin.argtypes = [ctypes.c_uint64]
    lib.oracle_msidx.restype = ctypes.c_uint32
    lib.oracle_msidx.argtypes = [ctypes.c_uint32] * 3
    lib.oracle_clean.restype = ctypes.c_int64
    lib.oracle_clean.argtypes = [ctypes.c_uint32, ctypes.c_uint64, p, p, p, p, p, p, p]
    lib.oracle_survey.restype = ctypes.c_int
    lib.oracle_survey.argtypes = [ctypes.c_uint32, ctypes.c_uint64, p, p, p, p, p,
                                  ctypes.POINTER(_Spec), ctypes.POINTER(_Result), ctypes.c_int,
                                  p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_max_edge_values.restype = ctypes.c_int
    lib.oracle_max_edge_values.argtypes = [ctypes.c_uint32, ctypes.c_uint64, p, p, p, p, ctypes.POINTER(_Spec),
                                           ctypes.POINTER(_Result), ctypes.c_int, p, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_directed_type.restype = ctypes.c_uint32
    lib.oracle_directed_type.argtypes = [ctypes.c_uint32] * 3
    lib.oracle_participation.restype = ctypes.c_int
    lib.oracle_participation.argtypes = [ctypes.c_uint32, ctypes.c_uint64, p, p, p, p, ctypes.POINTER(_Spec), p, p,
                                         ctypes.c_int]
    for f in ("oracle_sizeof_spec", "oracle_sizeof_result", "oracle_sizeof_tri"):
        getattr(lib, f).restype = ctypes.c_uint64
    assert lib.oracle_sizeof_spec() == ctypes.sizeof(_Spec)
    assert lib.oracle_sizeof_result() == ctypes.sizeof(_Result)
    assert lib.oracle_sizeof_tri() == TRI_DTYPE.itemsize
    _lib = lib
    return lib


def bin_of(d: int) -> int:
    return int(_load().oracle_bin(d))


def msidx(a: int, b: int, c: int) -> int:
    return int(_load().oracle_msidx(a, b, c))


def table_size(n_labels: int) -> int:
    L = n_labels
    return (L + 2) * (L + 1) * L // 6


def _ptr(a):
    return None if a is None else a.ctypes.data


def directed_type(d01: int, d02: int, d12: int) -> int:
    return int(_load().oracle_directed_type(d01, d02, d12))


def clean(n: int, src: np.ndarray, dst: np.ndarray, ts: np.ndarray | None, directions: bool = False):
    """Drop self-loops, keep each undirected pair once with its earliest time.
    Returns (u, v, t) with u < v, and with directions=True also the pair's
    direction bits (bit 0: u -> v occurs, bit 1: v -> u occurs)."""
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    ts = None if ts is None else np.ascontiguousarray(ts, np.uint32)
    M = len(src)
    u = np.empty(max(M, 1), np.uint32)
    v = np.empty(max(M, 1), np.uint32)
    t = np.empty(max(M, 1), np.uint32)
    d = np.zeros(max(M, 1), np.uint8) if directions else None
    m = _load().oracle_clean(n, M, _ptr(src), _ptr(dst), _ptr(ts), _ptr(u), _ptr(v), _ptr(t), _ptr(d))
    if m == -1:
        raise ValueError("vertex id out of range")
    if m < 0:
        raise MemoryError("oracle_clean")
    if directions:
        return u[:m].copy(), v[:m].copy(), t[:m].copy(), d[:m].copy()
    return u[:m].copy(), v[:m].copy(), t[:m].copy()


def survey_clean(n: int, u, v, t, vlab, outputs=("count",), n_labels: int = 4, spread_lt: int = 0,
                 window=None, label_mask=None, threads: int = 0, records: bool = False,
                 max_edge_shift: int = 0, edir=None):
    """Survey an already-cleaned graph.  Returns a dict of results (and the
    triangle records as a structured array when records=True)."""
    lib = _load()
    sp = _Spec()
    sp.outputs = sum(OUT_BITS[o] for o in outputs)
    sp.n_labels = n_labels
    sp.spread_lt = spread_lt
    sp.max_edge_shift = max_edge_shift
    if window is not None:
        sp.filters |= 1
        sp.t_lo, sp.t_hi = int(window[0]), int(window[1])
    if label_mask is not None:
        sp.filters |= 2
        for idx in label_mask:
            sp.label_mask[idx // 64] |= 1 << (idx % 64)
    res = _Result()
    u = np.ascontiguousarray(u, np.uint32)
    v = np.ascontiguousarray(v, np.uint32)
    t = np.ascontiguousarray(t, np.uint32)
    vlab = None if vlab is None else np.ascontiguousarray(vlab, np.uint8)
    edir = None if edir is None else np.ascontiguousarray(edir, np.uint8)
    recs = None
    cap = 0
    nrec = ctypes.c_uint64(0)
    if records:
        # first pass counts the triangles, second writes them
        rc = lib.oracle_survey(n, len(u), _ptr(u), _ptr(v), _ptr(t), _ptr(edir), _ptr(vlab), ctypes.byref(sp),
                               ctypes.byref(res), threads, None, 0, ctypes.byref(nrec))
        if rc != 0:
            raise RuntimeError("oracle_survey failed: %d" % rc)
        cap = res.triangles if (sp.filters == 0) else _count_all(lib, n, u, v, t, vlab, threads)
        recs = np.zeros(max(cap, 1), TRI_DTYPE)
        res = _Result()
    rc = lib.oracle_survey(n, len(u), _ptr(u), _ptr(v), _ptr(t), _ptr(edir), _ptr(vlab), ctypes.byref(sp),
                           ctypes.byref(res), threads, _ptr(recs), cap, ctypes.byref(nrec))
    if rc == -3:
        raise ValueError("vertex label >= n_labels")
    if rc == -4:
        raise ValueError("max_edge_shift must be below 32")
    if rc == -5:
        raise ValueError("the directed census needs the edge directions")
    if rc != 0:
        raise RuntimeError("oracle_survey failed: %d" % rc)
    out = dict(triangles=int(res.triangles), spread_count=int(res.spread_count),
               wedges=int(res.wedges),
               close_hist=np.frombuffer(bytes(res.close_hist), np.uint64).copy(),
               label_table=np.frombuffer(bytes(res.label_table), np.uint64)[:table_size(n_labels)].copy(),
               open_close=np.frombuffer(bytes(res.open_close), np.uint64).reshape(32, 32).copy(),
               max_edge=np.frombuffer(bytes(res.max_edge), np.uint64).copy(),
               degree_table=np.frombuffer(bytes(res.degree_table), np.uint64).copy(),
               directed=np.frombuffer(bytes(res.directed), np.uint64).copy())
    if records:
        out["records"] = recs[:int(nrec.value)]
    return out


def _count_all(lib, n, u, v, t, vlab, threads):
    sp = _Spec()
    sp.outputs = 1
    res = _Result()
    nrec = ctypes.c_uint64(0)
    lib.oracle_survey(n, len(u), _ptr(u), _ptr(v), _ptr(t), None, _ptr(vlab), ctypes.byref(sp),
                      ctypes.byref(res), threads, None, 0, ctypes.byref(nrec))
    return int(res.triangles)


def survey(n: int, src, dst, ts, vlab, **kw):
    """Clean the raw edge list, then survey it (the directed census reads
    the direction of every raw edge, src -> dst)."""
    if "directed" in kw.get("outputs", ()):
        u, v, t, d = clean(n, src, dst, ts, directions=True)
        kw["edir"] = d
    else:
        u, v, t = clean(n, src, dst, ts)
    out = survey_clean(n, u, v, t, vlab, **kw)
    out["m"] = len(u)
    return out


def max_edge_counts(n: int, src, dst, ts, vlab, n_labels: int = 4, window=None, label_mask=None,
                    threads: int = 0):
    """Algorithm 3's exact counting set (Section 4.5): over the triangles of
    the cleaned graph whose three vertex labels are pairwise distinct and
    that pass the filters (as in survey), every distinct largest edge time
    with its number of triangles.  Written from the definition: the largest
    time of every such triangle (oracle_max_edge_values, sized by the binned
    output's total), then numpy's unique to count equal values.  Returns
    (values ascending as uint32, counts as uint64)."""
    u, v, t = clean(n, src, dst, ts)
    kw = dict(n_labels=n_labels, window=window, label_mask=label_mask, threads=threads)
    total = int(survey_clean(n, u, v, t, vlab, outputs=("max_edge",), max_edge_shift=31, **kw)["max_edge"].sum())
    sp = _Spec()
    sp.n_labels = n_labels
    if window is not None:
        sp.filters |= 1
        sp.t_lo, sp.t_hi = int(window[0]), int(window[1])
    if label_mask is not None:
        sp.filters |= 2
        for idx in label_mask:
            sp.label_mask[idx // 64] |= 1 << (idx % 64)
    u, v, t = (np.ascontiguousarray(a, np.uint32) for a in (u, v, t))
    lab = np.ascontiguousarray(vlab, np.uint8)
    vals = np.zeros(max(total, 1), np.uint32)
    got = ctypes.c_uint64(0)
    res = _Result()
    rc = _load().oracle_max_edge_values(n, len(u), _ptr(u), _ptr(v), _ptr(t), _ptr(lab), ctypes.byref(sp),
                                        ctypes.byref(res), threads, _ptr(vals), total, ctypes.byref(got))
    if rc == -3:
        raise ValueError("vertex label >= n_labels")
    if rc != 0:
        raise RuntimeError("oracle_max_edge_values failed: %d" % rc)
    assert got.value == total
    vals, cnts = np.unique(vals[:total], return_counts=True)
    return vals.astype(np.uint32), cnts.astype(np.uint64)


def participation(n: int, src, dst, ts, vlab, n_labels: int = 4, window=None, label_mask=None, threads: int = 0):
    """Clean the raw edge list, then count the triangles at every vertex (by
    id) and at every edge.  Returns (vertex_counts, (u, v, t, edge_counts))
    with the cleaned edges sorted by (u, v), u < v."""
    u, v, t = clean(n, src, dst, ts)
    lib = _load()
    sp = _Spec()
    sp.n_labels = n_labels
    if window is not None:
        sp.filters |= 1
        sp.t_lo, sp.t_hi = int(window[0]), int(window[1])
    if label_mask is not None:
        sp.filters |= 2
        for idx in label_mask:
            sp.label_mask[idx // 64] |= 1 << (idx % 64)
    vlab = None if vlab is None else np.ascontiguousarray(vlab, np.uint8)
    vc = np.zeros(max(n, 1), np.uint64)
    ec = np.zeros(max(len(u), 1), np.uint64)
    rc = lib.oracle_participation(n, len(u), _ptr(u), _ptr(v), _ptr(t), _ptr(vlab), ctypes.byref(sp), _ptr(vc),
                                  _ptr(ec), threads)
    if rc == -3:
        raise ValueError("vertex label >= n_labels")
    if rc != 0:
        raise RuntimeError("oracle_participation failed: %d" % rc)
    return vc[:n], (u, v, t, ec[:len(u)])
