"""ctypes binding of libtripoll (include/tripoll.h): argument marshalling only.

Every function named ``tripoll_*`` here calls the C entry point of the same
name.  The helpers below them (``make_spec``, ``Graph``, ``build_graph``,
``survey``) only pack Python values into the C structs and unpack results;
all computation happens in the library's HIP kernels.  Loading fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtripoll.so")

# ------------------------------------------------------------------ constants
TP_OK, TP_ERR_INVALID, TP_ERR_OOM, TP_ERR_DEVICE, TP_ERR_BUSY, TP_ERR_UNSUPPORTED, TP_ERR_NOT_FOUND = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "OOM", 3: "DEVICE", 4: "BUSY", 5: "UNSUPPORTED", 6: "NOT_FOUND"}
TP_MEM_HOST, TP_MEM_DEVICE = 0, 1
TP_TIE_MIX, TP_TIE_ID = 0, 1
TP_OUT_COUNT, TP_OUT_CLOSE_HIST, TP_OUT_LABEL_TABLE, TP_OUT_SPREAD_COUNT, TP_OUT_OPEN_CLOSE = 1, 2, 4, 8, 16
TP_OUT_MAX_EDGE, TP_OUT_DEGREE_TABLE, TP_OUT_DIRECTED = 32, 64, 128
TP_EDGES_DIRECTED = 1
DIRECTED_TYPES = ("030T", "030C", "120D", "120U", "120C", "210", "300")
TP_FILT_WINDOW, TP_FILT_LABEL_MASK = 1, 2
TP_STRAT_AUTO, TP_STRAT_GLOBAL_SEARCH, TP_STRAT_TABLE_STRESS = 0, 1, 2
TP_VAR_DEFAULT, TP_VAR_WAVE_TABLE, TP_VAR_GROUP_TABLE, TP_VAR_SEARCH, TP_VAR_WAVE_SEARCH = 0, 1, 2, 3, 4
TP_NUM_CLASSES = 4
TP_MAX_LABELS = 16
TP_TABLE_MAX = 816
TP_MAX_EDGE_BINS = 1024
TP_DEGREE_MAX = 5984
TP_RW_TRIANGLES, TP_RW_SPREAD, TP_RW_PROBES, TP_RW_HIST = 0, 1, 2, 3
TP_RW_TABLE = TP_RW_HIST + 32
TP_RW_OPEN_CLOSE = TP_RW_TABLE + TP_TABLE_MAX
TP_RW_MAX_EDGE = TP_RW_OPEN_CLOSE + 1024
TP_RW_DEGREE = TP_RW_MAX_EDGE + TP_MAX_EDGE_BINS
TP_RW_DIRECTED = TP_RW_DEGREE + TP_DEGREE_MAX
TP_RW_SCRATCH = TP_RW_DIRECTED + 8
TP_RW_CLASS_TRI = TP_RW_SCRATCH + 4
TP_RESULT_WORDS = TP_RW_SCRATCH + 16
TP_BW_TRIANGLES, TP_BW_SPREAD, TP_BW_PROBES, TP_BW_HIST, TP_BW_TABLE = 0, 1, 2, 3, 35
TP_BATCH_SCRATCH_WORDS = 8

OUT_BITS = {"count": TP_OUT_COUNT, "close_hist": TP_OUT_CLOSE_HIST, "label_table": TP_OUT_LABEL_TABLE,
            "spread_count": TP_OUT_SPREAD_COUNT, "open_close": TP_OUT_OPEN_CLOSE,
            "max_edge": TP_OUT_MAX_EDGE, "degree_table": TP_OUT_DEGREE_TABLE, "directed": TP_OUT_DIRECTED}


class tp_edge_list(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint32), ("mem_space", ctypes.c_uint32), ("n_edges", ctypes.c_uint64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("edge_time", ctypes.c_void_p),
                ("vertex_label", ctypes.c_void_p), ("tie_hash", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class tp_batch_edges(ctypes.Structure):
    _fields_ = [("n_graphs", ctypes.c_uint32), ("mem_space", ctypes.c_uint32), ("edge_offsets", ctypes.c_void_p),
                ("vertex_counts", ctypes.c_void_p), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("edge_time", ctypes.c_void_p), ("vertex_label", ctypes.c_void_p), ("tie_hash", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class tp_graph_stats(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint64), ("n_raw_edges", ctypes.c_uint64),
                ("n_self_loops", ctypes.c_uint64), ("n_edges", ctypes.c_uint64), ("d_max", ctypes.c_uint64),
                ("dplus_max", ctypes.c_uint64), ("wedges", ctypes.c_uint64), ("probes", ctypes.c_uint64),
                ("n_targets", ctypes.c_uint64), ("n_tiles", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("max_label", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("phase_ms", ctypes.c_float * 8), ("build_ms", ctypes.c_float), ("reserved2", ctypes.c_uint32),
                ("class_tiles", ctypes.c_uint64 * TP_NUM_CLASSES), ("class_records", ctypes.c_uint64 * TP_NUM_CLASSES),
                ("class_staged", ctypes.c_uint64 * TP_NUM_CLASSES), ("class_probes", ctypes.c_uint64 * TP_NUM_CLASSES)]


class tp_survey_spec(ctypes.Structure):
    _fields_ = [("outputs", ctypes.c_uint32), ("filters", ctypes.c_uint32), ("n_labels", ctypes.c_uint32),
                ("strategy", ctypes.c_uint32), ("spread_lt", ctypes.c_uint64), ("t_lo", ctypes.c_uint64),
                ("t_hi", ctypes.c_uint64), ("label_mask", ctypes.c_uint64 * 13),
                ("max_edge_shift", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class tp_survey_result(ctypes.Structure):
    _fields_ = [("triangles", ctypes.c_uint64), ("spread_count", ctypes.c_uint64), ("probes", ctypes.c_uint64),
                ("close_hist", ctypes.c_uint64 * 32), ("label_table", ctypes.c_uint64 * TP_TABLE_MAX),
                ("open_close", ctypes.c_uint64 * 1024), ("max_edge", ctypes.c_uint64 * TP_MAX_EDGE_BINS),
                ("degree_table", ctypes.c_uint64 * TP_DEGREE_MAX), ("directed", ctypes.c_uint64 * 8),
                ("kernel_ms", ctypes.c_float),
                ("total_ms", ctypes.c_float), ("class_ms", ctypes.c_float * TP_NUM_CLASSES),
                ("class_triangles", ctypes.c_uint64 * TP_NUM_CLASSES)]


class tp_plan(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_uint32 * TP_NUM_CLASSES), ("tile_records", ctypes.c_uint32 * TP_NUM_CLASSES)]


class tp_tune_result(ctypes.Structure):
    _fields_ = [("chosen", tp_plan), ("default_ms", ctypes.c_float * TP_NUM_CLASSES),
                ("tuned_ms", ctypes.c_float * TP_NUM_CLASSES), ("trials", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


TP_SERVER_TAGS = 8


class tp_server_config(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_uint32), ("n_labels", ctypes.c_uint32), ("hbm_budget", ctypes.c_uint64),
                ("step_wedges", ctypes.c_uint64), ("max_queue", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class tp_request_info(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint32), ("steps", ctypes.c_uint32), ("arrival_us", ctypes.c_double),
                ("admit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class tp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("waiting", ctypes.c_uint64), ("running", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("triangles", ctypes.c_uint64), ("hbm_used", ctypes.c_uint64), ("hbm_budget", ctypes.c_uint64),
                ("elapsed_s", ctypes.c_double), ("count", ctypes.c_uint64 * TP_SERVER_TAGS),
                ("p50_ms", ctypes.c_double * TP_SERVER_TAGS), ("p99_ms", ctypes.c_double * TP_SERVER_TAGS)]


class TripollError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None

# symbol -> (restype, argtypes)
_P = ctypes.c_void_p
SIGNATURES = {
    "tripoll_build": (ctypes.c_int, [ctypes.POINTER(tp_edge_list), _P, ctypes.POINTER(_P)]),
    "tripoll_graph_stats": (ctypes.c_int, [_P, ctypes.POINTER(tp_graph_stats)]),
    "tripoll_graph_free": (ctypes.c_int, [_P]),
    "tripoll_graph_export": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "tripoll_survey": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), ctypes.POINTER(tp_survey_result), _P]),
    "tripoll_survey_async": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, _P]),
    "tripoll_survey_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), ctypes.POINTER(tp_survey_result),
                                              _P]),
    "tripoll_max_edge_counts": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, _P, ctypes.c_uint64,
                                               ctypes.POINTER(ctypes.c_uint64), _P]),
    "tripoll_enumerate": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), _P]),
    "tripoll_participation": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, _P,
                                             ctypes.POINTER(ctypes.c_uint64), _P]),
    "tripoll_enum_open": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, ctypes.POINTER(_P),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    "tripoll_enum_next": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), _P]),
    "tripoll_enum_close": (ctypes.c_int, [_P]),
    "tripoll_build_batch": (ctypes.c_int, [ctypes.POINTER(tp_batch_edges), _P, ctypes.POINTER(_P)]),
    "tripoll_graph_count": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32)]),
    "tripoll_batch_words": (ctypes.c_uint64, [ctypes.POINTER(tp_survey_spec)]),
    "tripoll_survey_batch": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, _P]),
    "tripoll_survey_capture": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, ctypes.POINTER(_P)]),
    "tripoll_launch_replay": (ctypes.c_int, [_P, _P]),
    "tripoll_launch_free": (ctypes.c_int, [_P]),
    "tripoll_get_plan": (ctypes.c_int, [_P, ctypes.POINTER(tp_plan)]),
    "tripoll_set_plan": (ctypes.c_int, [_P, ctypes.POINTER(tp_plan), _P]),
    "tripoll_tune": (ctypes.c_int, [_P, ctypes.POINTER(tp_survey_spec), _P, ctypes.POINTER(tp_tune_result)]),
    "tripoll_server_create": (ctypes.c_int, [ctypes.POINTER(tp_server_config), ctypes.POINTER(_P)]),
    "tripoll_server_destroy": (ctypes.c_int, [_P]),
    "tripoll_server_add_graph": (ctypes.c_int, [_P, ctypes.POINTER(tp_edge_list), ctypes.POINTER(ctypes.c_uint32)]),
    "tripoll_server_remove_graph": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "tripoll_server_graph_stats": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(tp_graph_stats)]),
    "tripoll_server_graph": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "tripoll_server_submit": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(tp_survey_spec), ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "tripoll_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(tp_survey_result),
                                           ctypes.POINTER(tp_request_info)]),
    "tripoll_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(tp_server_stats)]),
    "tripoll_msidx": (ctypes.c_uint32, [ctypes.c_uint32] * 3),
    "tripoll_trim": (ctypes.c_int, []),
    "tripoll_cached_bytes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64)]),
    "tripoll_live_bytes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64)]),
    "tripoll_fail_alloc_after": (ctypes.c_int, [ctypes.c_uint64]),
    "tripoll_last_error": (ctypes.c_char_p, []),
    "tripoll_version": (ctypes.c_char_p, []),
}


def load():
    """Load libtripoll.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtripoll.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != TP_OK:
        raise TripollError(status, load().tripoll_last_error().decode())


# ------------------------------------------------------------------ raw entry points

def tripoll_build(edges: tp_edge_list, stream=None) -> int:
    g = _P()
    _check(load().tripoll_build(ctypes.byref(edges), stream, ctypes.byref(g)))
    return g.value


def tripoll_graph_stats(g: int) -> tp_graph_stats:
    st = tp_graph_stats()
    _check(load().tripoll_graph_stats(g, ctypes.byref(st)))
    return st


def tripoll_graph_free(g: int) -> None:
    _check(load().tripoll_graph_free(g))


def tripoll_graph_export(g, rowptr=None, col=None, etime=None, tlabel=None, rank_to_id=None, rank_label=None):
    ptr = lambda a: None if a is None else a.ctypes.data
    _check(load().tripoll_graph_export(g, ptr(rowptr), ptr(col), ptr(etime), ptr(tlabel), ptr(rank_to_id),
                                       ptr(rank_label)))


def tripoll_survey(g: int, spec: tp_survey_spec, stream=None) -> tp_survey_result:
    res = tp_survey_result()
    _check(load().tripoll_survey(g, ctypes.byref(spec), ctypes.byref(res), stream))
    return res


def tripoll_survey_noalloc(g: int, spec: tp_survey_spec, stream=None) -> tp_survey_result:
    res = tp_survey_result()
    _check(load().tripoll_survey_noalloc(g, ctypes.byref(spec), ctypes.byref(res), stream))
    return res


def tripoll_survey_async(g: int, spec: tp_survey_spec, dev_out: int, stream=None) -> None:
    _check(load().tripoll_survey_async(g, ctypes.byref(spec), dev_out, stream))


def tripoll_max_edge_counts(g: int, spec: tp_survey_spec, dev_values: int, dev_counts: int, capacity: int,
                            stream=None) -> int:
    """Number of distinct values written; on TP_ERR_INVALID for a too small
    capacity the error's n_values holds the number needed."""
    n = ctypes.c_uint64(0)
    st = load().tripoll_max_edge_counts(g, ctypes.byref(spec), dev_values, dev_counts, capacity, ctypes.byref(n),
                                        stream)
    if st != TP_OK:
        err = TripollError(st, load().tripoll_last_error().decode())
        err.n_values = n.value
        raise err
    return n.value


def tripoll_enumerate(g: int, dev_records: int, capacity: int, stream=None) -> int:
    n = ctypes.c_uint64(0)
    _check(load().tripoll_enumerate(g, dev_records, capacity, ctypes.byref(n), stream))
    return n.value


def tripoll_build_batch(batch: tp_batch_edges, stream=None) -> int:
    g = _P()
    _check(load().tripoll_build_batch(ctypes.byref(batch), stream, ctypes.byref(g)))
    return g.value


def tripoll_graph_count(g: int) -> int:
    v = ctypes.c_uint32(0)
    _check(load().tripoll_graph_count(g, ctypes.byref(v)))
    return v.value


def tripoll_enum_open(g: int, spec: tp_survey_spec, stream=None) -> tuple:
    """Open a streamed enumeration; returns (handle, total records, records
    of the largest tile)."""
    h = _P()
    total, mx = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().tripoll_enum_open(g, ctypes.byref(spec), stream, ctypes.byref(h), ctypes.byref(total),
                                    ctypes.byref(mx)))
    return h.value, int(total.value), int(mx.value)


def tripoll_enum_next(e: int, dev_records: int, capacity: int, stream=None) -> int:
    n = ctypes.c_uint64(0)
    _check(load().tripoll_enum_next(e, dev_records, capacity, ctypes.byref(n), stream))
    return int(n.value)


def tripoll_enum_close(e: int) -> None:
    _check(load().tripoll_enum_close(e))


def tripoll_participation(g: int, spec: tp_survey_spec, vertex_counts: int, edge_counts: int, stream=None) -> int:
    """Per-vertex and per-edge triangle counts into device buffers (either
    pointer may be 0); returns the number of triangles counted."""
    tri = ctypes.c_uint64(0)
    _check(load().tripoll_participation(g, ctypes.byref(spec), vertex_counts or None, edge_counts or None,
                                        ctypes.byref(tri), stream))
    return int(tri.value)


def tripoll_batch_words(spec: tp_survey_spec) -> int:
    return int(load().tripoll_batch_words(ctypes.byref(spec)))


def tripoll_survey_batch(g: int, spec: tp_survey_spec, dev_out: int, stream=None) -> None:
    _check(load().tripoll_survey_batch(g, ctypes.byref(spec), dev_out, stream))


def tripoll_survey_capture(g: int, spec: tp_survey_spec, dev_out: int) -> int:
    h = _P()
    _check(load().tripoll_survey_capture(g, ctypes.byref(spec), dev_out, ctypes.byref(h)))
    return h.value


def tripoll_launch_replay(launch: int, stream=None) -> None:
    _check(load().tripoll_launch_replay(launch, stream))


def tripoll_launch_free(launch: int) -> None:
    _check(load().tripoll_launch_free(launch))


def tripoll_get_plan(g: int) -> tp_plan:
    p = tp_plan()
    _check(load().tripoll_get_plan(g, ctypes.byref(p)))
    return p


def tripoll_set_plan(g: int, plan: tp_plan, stream=None) -> None:
    _check(load().tripoll_set_plan(g, ctypes.byref(plan), stream))


def tripoll_tune(g: int, spec: tp_survey_spec, stream=None) -> tp_tune_result:
    r = tp_tune_result()
    _check(load().tripoll_tune(g, ctypes.byref(spec), stream, ctypes.byref(r)))
    return r


def tripoll_server_create(cfg: tp_server_config) -> int:
    h = _P()
    _check(load().tripoll_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def tripoll_server_destroy(srv: int) -> None:
    _check(load().tripoll_server_destroy(srv))


def tripoll_server_add_graph(srv: int, edges: tp_edge_list) -> int:
    gid = ctypes.c_uint32(0)
    _check(load().tripoll_server_add_graph(srv, ctypes.byref(edges), ctypes.byref(gid)))
    return gid.value


def tripoll_server_remove_graph(srv: int, graph_id: int) -> None:
    _check(load().tripoll_server_remove_graph(srv, graph_id))


def tripoll_server_graph_stats(srv: int, graph_id: int) -> tp_graph_stats:
    st = tp_graph_stats()
    _check(load().tripoll_server_graph_stats(srv, graph_id, ctypes.byref(st)))
    return st


def tripoll_server_graph(srv: int, graph_id: int) -> int:
    h = _P()
    _check(load().tripoll_server_graph(srv, graph_id, ctypes.byref(h)))
    return h.value


def tripoll_server_submit(srv: int, graph_id: int, spec: tp_survey_spec, tag: int = 0) -> int:
    t = ctypes.c_uint64(0)
    _check(load().tripoll_server_submit(srv, graph_id, ctypes.byref(spec), tag, ctypes.byref(t)))
    return t.value


def tripoll_server_wait(srv: int, ticket: int, timeout_us: int = -1):
    res = tp_survey_result()
    info = tp_request_info()
    _check(load().tripoll_server_wait(srv, ticket, timeout_us, ctypes.byref(res), ctypes.byref(info)))
    return res, info


def tripoll_server_stats(srv: int) -> tp_server_stats:
    st = tp_server_stats()
    _check(load().tripoll_server_stats(srv, ctypes.byref(st)))
    return st


def tripoll_msidx(a: int, b: int, c: int) -> int:
    return int(load().tripoll_msidx(a, b, c))


def tripoll_trim() -> None:
    _check(load().tripoll_trim())


def tripoll_cached_bytes() -> int:
    v = ctypes.c_uint64(0)
    _check(load().tripoll_cached_bytes(ctypes.byref(v)))
    return v.value


def tripoll_live_bytes() -> int:
    v = ctypes.c_uint64(0)
    _check(load().tripoll_live_bytes(ctypes.byref(v)))
    return v.value


def tripoll_fail_alloc_after(n: int) -> None:
    _check(load().tripoll_fail_alloc_after(n))


def tripoll_version() -> str:
    return load().tripoll_version().decode()


# ------------------------------------------------------------------ marshalling helpers

def table_size(n_labels: int) -> int:
    return (n_labels + 2) * (n_labels + 1) * n_labels // 6


def make_spec(outputs=("count",), n_labels=4, spread_lt=0, window=None, label_mask=None,
              strategy=TP_STRAT_AUTO, max_edge_shift=0) -> tp_survey_spec:
    sp = tp_survey_spec()
    sp.outputs = sum(OUT_BITS[o] for o in outputs)
    sp.n_labels = n_labels
    sp.strategy = strategy
    sp.spread_lt = spread_lt
    sp.max_edge_shift = max_edge_shift
    if window is not None:
        sp.filters |= TP_FILT_WINDOW
        sp.t_lo, sp.t_hi = int(window[0]), int(window[1])
    if label_mask is not None:
        sp.filters |= TP_FILT_LABEL_MASK
        for idx in label_mask:
            sp.label_mask[idx // 64] |= 1 << (idx % 64)
    return sp


def result_dict(res: tp_survey_result, n_labels: int = 16) -> dict:
    return dict(triangles=int(res.triangles), spread_count=int(res.spread_count), probes=int(res.probes),
                close_hist=np.frombuffer(bytes(res.close_hist), np.uint64).copy(),
                label_table=np.frombuffer(bytes(res.label_table), np.uint64)[:table_size(n_labels)].copy(),
                open_close=np.frombuffer(bytes(res.open_close), np.uint64).reshape(32, 32).copy(),
                max_edge=np.frombuffer(bytes(res.max_edge), np.uint64).copy(),
                degree_table=np.frombuffer(bytes(res.degree_table), np.uint64).copy(),
                directed=np.frombuffer(bytes(res.directed), np.uint64)[:7].copy(),
                kernel_ms=float(res.kernel_ms), total_ms=float(res.total_ms),
                class_ms=[float(x) for x in res.class_ms],
                class_triangles=[int(x) for x in res.class_triangles])


def words_dict(words: np.ndarray, n_labels: int = 16) -> dict:
    """Unpack a device result buffer (TP_RESULT_WORDS uint64) copied to host."""
    w = np.asarray(words, np.uint64)
    return dict(triangles=int(w[TP_RW_TRIANGLES]), spread_count=int(w[TP_RW_SPREAD]),
                probes=int(w[TP_RW_PROBES]), close_hist=w[TP_RW_HIST:TP_RW_HIST + 32].copy(),
                label_table=w[TP_RW_TABLE:TP_RW_TABLE + table_size(n_labels)].copy(),
                open_close=w[TP_RW_OPEN_CLOSE:TP_RW_OPEN_CLOSE + 1024].reshape(32, 32).copy(),
                max_edge=w[TP_RW_MAX_EDGE:TP_RW_MAX_EDGE + TP_MAX_EDGE_BINS].copy(),
                degree_table=w[TP_RW_DEGREE:TP_RW_DEGREE + TP_DEGREE_MAX].copy(),
                directed=w[TP_RW_DIRECTED:TP_RW_DIRECTED + 7].copy())


def stats_dict(st: tp_graph_stats) -> dict:
    d = {f: getattr(st, f) for f, _ in tp_graph_stats._fields_ if not f.startswith(("phase_ms", "reserved", "class_"))}
    d["phase_ms"] = list(st.phase_ms)
    for f in ("class_tiles", "class_records", "class_staged", "class_probes"):
        d[f] = [int(x) for x in getattr(st, f)]
    return d


def _addr(a):
    """Address of a numpy array or a torch tensor (host or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return int(a.data_ptr())


def edge_list(n, src, dst, ts=None, vlab=None, tie=TP_TIE_MIX, device=None, directed=False) -> tp_edge_list:
    """Pack arrays into a tp_edge_list.  `device` True for device tensors;
    by default inferred from the arrays (numpy = host).  directed=True keeps
    the direction src -> dst of every edge for the directed census."""
    if device is None:
        device = not isinstance(src, np.ndarray)
    el = tp_edge_list()
    el.n_vertices = n
    el.mem_space = TP_MEM_DEVICE if device else TP_MEM_HOST
    el.n_edges = len(src)
    el.src, el.dst, el.edge_time, el.vertex_label = _addr(src), _addr(dst), _addr(ts), _addr(vlab)
    el.tie_hash = tie
    el.flags = TP_EDGES_DIRECTED if directed else 0
    return el


class Graph:
    """Owning handle of a built graph (released by close() or on exit)."""

    def __init__(self, handle: int):
        self.handle = handle

    def stats(self) -> dict:
        return stats_dict(tripoll_graph_stats(self.handle))

    def close(self):
        if self.handle:
            tripoll_graph_free(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_graph(n, src, dst, ts=None, vlab=None, tie=TP_TIE_MIX, stream=None, directed=False) -> Graph:
    return Graph(tripoll_build(edge_list(n, src, dst, ts, vlab, tie, directed=directed), stream))


def survey(graph: Graph, stream=None, n_labels=4, **spec_kw) -> dict:
    res = tripoll_survey(graph.handle, make_spec(n_labels=n_labels, **spec_kw), stream)
    return result_dict(res, n_labels)


def max_edge_counts(graph: Graph, torch, stream=None, **spec_kw):
    """Algorithm 3's exact counting set of a graph as (values, counts) numpy
    arrays, values ascending; device buffers of m entries (enough for any
    graph) come from torch."""
    spec = make_spec(**spec_kw)
    m = max(1, graph.stats()["n_edges"])
    vals = torch.empty(m, dtype=torch.int32, device="cuda")
    cnts = torch.empty(m, dtype=torch.int64, device="cuda")
    n = tripoll_max_edge_counts(graph.handle, spec, vals.data_ptr(), cnts.data_ptr(), m, stream)
    return (vals[:n].cpu().numpy().view(np.uint32).copy(), cnts[:n].cpu().numpy().view(np.uint64).copy())


def export(graph: Graph) -> dict:
    st = graph.stats()
    n, m = st["n_vertices"], st["n_edges"]
    out = dict(rowptr=np.empty(n + 1, np.uint64), col=np.empty(m, np.uint32), etime=np.empty(m, np.uint32),
               tlabel=np.empty(m, np.uint8), rank_to_id=np.empty(n, np.uint32), rank_label=np.empty(n, np.uint8))
    tripoll_graph_export(graph.handle, **out)
    return out


# ------------------------------------------------------------------ batches

def batch_edges(edge_offsets, vertex_counts, src, dst, ts=None, vlab=None, tie=TP_TIE_MIX,
                device=None, directed=False) -> tuple:
    """Pack a batch into a tp_batch_edges.  Returns (struct, keep-alive host
    arrays); the offsets and counts are always host arrays.  directed=True
    keeps every edge's direction src -> dst for the directed census."""
    if device is None:
        device = not isinstance(src, np.ndarray)
    eoff = np.ascontiguousarray(edge_offsets, np.uint64)
    vcnt = np.ascontiguousarray(vertex_counts, np.uint32)
    be = tp_batch_edges()
    be.n_graphs = len(vcnt)
    be.mem_space = TP_MEM_DEVICE if device else TP_MEM_HOST
    be.edge_offsets, be.vertex_counts = eoff.ctypes.data, vcnt.ctypes.data
    be.src, be.dst, be.edge_time, be.vertex_label = _addr(src), _addr(dst), _addr(ts), _addr(vlab)
    be.tie_hash = tie
    be.flags = TP_EDGES_DIRECTED if directed else 0
    return be, (eoff, vcnt)


def build_batch(edge_offsets, vertex_counts, src, dst, ts=None, vlab=None, tie=TP_TIE_MIX, stream=None,
                directed=False) -> Graph:
    be, keep = batch_edges(edge_offsets, vertex_counts, src, dst, ts, vlab, tie, directed=directed)
    h = tripoll_build_batch(be, stream)
    del keep
    return Graph(h)


def batch_dicts(words: np.ndarray, n_graphs: int, spec: tp_survey_spec, n_labels: int) -> list:
    """Unpack the per-graph blocks of a batch result copied to host."""
    bw = tripoll_batch_words(spec)
    w = np.asarray(words, np.uint64)[:n_graphs * bw].reshape(n_graphs, bw)
    ts = table_size(n_labels) if spec.outputs & TP_OUT_LABEL_TABLE else 0
    oc = TP_BW_TABLE + ts
    out = []
    for g in range(n_graphs):
        r = w[g]
        d = dict(triangles=int(r[TP_BW_TRIANGLES]), spread_count=int(r[TP_BW_SPREAD]), probes=int(r[TP_BW_PROBES]),
                 close_hist=r[TP_BW_HIST:TP_BW_HIST + 32].copy())
        if ts:
            d["label_table"] = r[TP_BW_TABLE:TP_BW_TABLE + ts].copy()
        at = oc
        if spec.outputs & TP_OUT_OPEN_CLOSE:
            d["open_close"] = r[at:at + 1024].reshape(32, 32).copy()
            at += 1024
        if spec.outputs & TP_OUT_MAX_EDGE:
            d["max_edge"] = r[at:at + TP_MAX_EDGE_BINS].copy()
            at += TP_MAX_EDGE_BINS
        if spec.outputs & TP_OUT_DEGREE_TABLE:
            d["degree_table"] = r[at:at + TP_DEGREE_MAX].copy()
            at += TP_DEGREE_MAX
        if spec.outputs & TP_OUT_DIRECTED:
            d["directed"] = r[at:at + 7].copy()
            at += 8
        out.append(d)
    return out


class Launch:
    """Owning handle of a recorded survey launch."""

    def __init__(self, handle: int):
        self.handle = handle

    def replay(self, stream=None):
        tripoll_launch_replay(self.handle, stream)

    def close(self):
        if self.handle:
            tripoll_launch_free(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ plans

def make_plan(variants=(TP_VAR_DEFAULT,) * TP_NUM_CLASSES, tile_records=(1024,) * TP_NUM_CLASSES) -> tp_plan:
    p = tp_plan()
    for i in range(TP_NUM_CLASSES):
        p.variant[i] = variants[i]
        p.tile_records[i] = tile_records[i]
    return p


def plan_dict(p: tp_plan) -> dict:
    return dict(variant=[int(x) for x in p.variant], tile_records=[int(x) for x in p.tile_records])


def tune_dict(r: tp_tune_result) -> dict:
    return dict(chosen=plan_dict(r.chosen), default_ms=[round(float(x), 3) for x in r.default_ms],
                tuned_ms=[round(float(x), 3) for x in r.tuned_ms], trials=int(r.trials))


# ------------------------------------------------------------------ served mode

class Server:
    """Owning handle of a survey server (tripoll_server_*)."""

    def __init__(self, max_slots=8, n_labels=8, hbm_budget=0, step_wedges=0, max_queue=0):
        cfg = tp_server_config()
        cfg.max_slots, cfg.n_labels, cfg.hbm_budget = max_slots, n_labels, hbm_budget
        cfg.step_wedges, cfg.max_queue = step_wedges, max_queue
        self.n_labels = n_labels
        self.handle = tripoll_server_create(cfg)

    def add_graph(self, n, src, dst, ts=None, vlab=None, tie=TP_TIE_MIX, directed=False) -> int:
        return tripoll_server_add_graph(self.handle, edge_list(n, src, dst, ts, vlab, tie, directed=directed))

    def remove_graph(self, graph_id: int):
        tripoll_server_remove_graph(self.handle, graph_id)

    def graph_stats(self, graph_id: int) -> dict:
        return stats_dict(tripoll_server_graph_stats(self.handle, graph_id))

    def graph(self, graph_id: int) -> int:
        """Borrowed tp_graph handle of a resident graph."""
        return tripoll_server_graph(self.handle, graph_id)

    def submit(self, graph_id: int, tag: int = 0, **spec_kw) -> int:
        spec_kw.setdefault("n_labels", self.n_labels)
        return tripoll_server_submit(self.handle, graph_id, make_spec(**spec_kw), tag)

    def wait(self, ticket: int, timeout_us: int = -1) -> tuple:
        res, info = tripoll_server_wait(self.handle, ticket, timeout_us)
        d = result_dict(res, self.n_labels)
        return d, dict(tag=int(info.tag), steps=int(info.steps), arrival_us=info.arrival_us,
                       admit_us=info.admit_us, done_us=info.done_us)

    def stats(self) -> dict:
        st = tripoll_server_stats(self.handle)
        d = {f: getattr(st, f) for f, _ in tp_server_stats._fields_ if f not in ("count", "p50_ms", "p99_ms")}
        for f in ("count", "p50_ms", "p99_ms"):
            d[f] = list(getattr(st, f))
        return d

    def close(self):
        if self.handle:
            tripoll_server_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
