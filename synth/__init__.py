"""Seeded synthetic inputs for the triangle survey (edge lists, edge
timestamps, vertex labels, batch parameters).

This module produces raw inputs only and holds none of the survey's
arithmetic.  Both the CPU oracle tests and the GPU path take their inputs
from here, so the two sides see identical bytes.  The generator itself is
plain C (``tpgen.c``) driven through ctypes; every value is a function of
(seed, stream, index) only.

Workloads follow the paper's synthetic family: R-MAT graphs (Evaluation,
Datasets and Weak Scaling subsections) with a=0.57, b=0.19, c=0.19, d=0.05,
edge factor 16, undirected; edge timestamps as edge metadata (the Reddit
closure-time study) and small integer vertex labels (the labelled-triangle
examples of the Callback Examples subsection).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpgen.c")
_LIB = os.path.join(_HERE, "libtpgen.so")
_DEV_SRC = os.path.join(_HERE, "tpgen_dev.hip")
_DEV_LIB = os.path.join(_HERE, "libtpgen_dev.so")

# R-MAT quadrant thresholds floor(p * 2^32) for a=0.57, a+b=0.76, a+b+c=0.95.
RMAT_THR = ((57 << 32) // 100, (76 << 32) // 100, (95 << 32) // 100)
# Zipf(s=1.2) over labels 0..7: cumulative thresholds floor(CDF_k * 2^32),
# k = 0..6, with p_k proportional to (k+1)^-1.2.
ZIPF12_L8_THR = (1840948827, 2642268346, 3134870392, 3483664971,
                 3750521426, 3964938920, 4143145637)
MASTER_SEED = 2107123300

_lib = None


def build(verbose: bool = False) -> str:
    """Compile libtpgen.so with gcc (OpenMP) and the device batch generator
    libtpgen_dev.so with hipcc for gfx950."""
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", _DEV_LIB + ".tmp", _DEV_SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_DEV_LIB + ".tmp", _DEV_LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    lib.tpgen_draw.restype = u64
    lib.tpgen_draw.argtypes = [u64, u32, u64]
    lib.tpgen_rmat.argtypes = [u64, u32, u64, u32, u32, u32, p, p]
    lib.tpgen_er.argtypes = [u64, u32, u64, p, p]
    lib.tpgen_ts_uniform.argtypes = [u64, u64, u32, p]
    lib.tpgen_ts_bursty.argtypes = [u64, u64, u32, p]
    lib.tpgen_labels_uniform.argtypes = [u64, u32, u32, p]
    lib.tpgen_labels_cdf.argtypes = [u64, u32, p, u32, p]
    lib.tpgen_batch_params.argtypes = [u64, u32, u32, u32, u32, u32,
                                       ctypes.POINTER(u64), ctypes.POINTER(u32),
                                       ctypes.POINTER(u32), ctypes.POINTER(u32)]
    _lib = lib
    return lib


def draw(seed: int, stream: int, index: int) -> int:
    return int(_load().tpgen_draw(seed, stream, index))


@dataclass
class GraphSpec:
    """Recipe of one synthetic graph."""
    kind: str = "rmat"          # "rmat" | "er"
    scale: int = 12             # n = 2^scale vertices
    edge_factor: int = 16       # raw edges = edge_factor * n
    seed: int = MASTER_SEED
    ts: tuple = ("uniform", 20)     # ("uniform", bits) | ("bursty", n_bursts) | ("zero",)
    labels: tuple = ("uniform", 4)  # ("uniform", L) | ("zipf12", 8) | ("zero",)

    @property
    def n(self) -> int:
        return 1 << self.scale

    @property
    def n_edges(self) -> int:
        return self.edge_factor << self.scale


def _ptr(a) -> int:
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return int(a)


def fill_edges(spec: GraphSpec, src, dst) -> None:
    """Write the spec's raw edges into src/dst (numpy arrays or host pointers)."""
    lib = _load()
    if spec.kind == "rmat":
        lib.tpgen_rmat(spec.seed, spec.scale, spec.n_edges, *RMAT_THR, _ptr(src), _ptr(dst))
    elif spec.kind == "er":
        lib.tpgen_er(spec.seed, spec.n, spec.n_edges, _ptr(src), _ptr(dst))
    else:
        raise ValueError(spec.kind)


def fill_ts(spec: GraphSpec, ts) -> None:
    lib = _load()
    kind = spec.ts[0]
    if kind == "uniform":
        lib.tpgen_ts_uniform(spec.seed, spec.n_edges, spec.ts[1], _ptr(ts))
    elif kind == "bursty":
        lib.tpgen_ts_bursty(spec.seed, spec.n_edges, spec.ts[1], _ptr(ts))
    elif kind == "zero":
        ctypes.memset(_ptr(ts), 0, 4 * spec.n_edges)
    else:
        raise ValueError(kind)


def fill_labels(spec: GraphSpec, lab) -> None:
    lib = _load()
    kind = spec.labels[0]
    if kind == "uniform":
        lib.tpgen_labels_uniform(spec.seed, spec.n, spec.labels[1], _ptr(lab))
    elif kind == "zipf12":
        thr = (ctypes.c_uint32 * 7)(*ZIPF12_L8_THR)
        lib.tpgen_labels_cdf(spec.seed, spec.n, ctypes.addressof(thr), 8, _ptr(lab))
    elif kind == "zero":
        ctypes.memset(_ptr(lab), 0, spec.n)
    else:
        raise ValueError(kind)


def n_labels(spec: GraphSpec) -> int:
    return 1 if spec.labels[0] == "zero" else int(spec.labels[1])


def generate(spec: GraphSpec) -> dict:
    """Return numpy arrays src, dst, ts (uint32[M]) and vlab (uint8[n])."""
    M, n = spec.n_edges, spec.n
    src = np.empty(M, np.uint32)
    dst = np.empty(M, np.uint32)
    ts = np.empty(M, np.uint32)
    vlab = np.empty(n, np.uint8)
    fill_edges(spec, src, dst)
    fill_ts(spec, ts)
    fill_labels(spec, vlab)
    return dict(n=n, src=src, dst=dst, ts=ts, vlab=vlab)


# --------------------------------------------------------------------------
# The five workloads.  Survey outputs are named by plain strings here; the
# binding and the oracle wrapper each translate them into their own form.
# --------------------------------------------------------------------------

@dataclass
class Workload:
    number: int
    name: str
    graph: GraphSpec | None
    outputs: tuple = ()
    n_labels: int = 4
    spread_lt: int = 0
    extra: dict = field(default_factory=dict)


def workload(number: int, scale: int | None = None) -> Workload:
    """Workload 1..5.  `scale` overrides the graph scale (same recipe)."""
    seed = MASTER_SEED + number
    if number == 1:
        g = GraphSpec("rmat", scale or 12, 16, seed, ("uniform", 20), ("uniform", 4))
        return Workload(1, "rmat-s%d-uniform" % g.scale, g, ("count", "close_hist", "label_table"), 4)
    if number == 2:
        g = GraphSpec("rmat", scale or 22, 16, seed, ("uniform", 30), ("zipf12", 8))
        return Workload(2, "rmat-s%d-zipf" % g.scale, g, ("count", "close_hist", "label_table"), 8)
    if number == 3:
        g = GraphSpec("rmat", scale or 26, 16, seed, ("bursty", 64), ("uniform", 4))
        return Workload(3, "rmat-s%d-bursty" % g.scale, g,
                        ("count", "close_hist", "label_table", "spread_count"), 4, spread_lt=1 << 16)
    if number == 4:
        return Workload(4, "batch-20000", None, ("count", "close_hist"), 8,
                        extra=dict(n_graphs=20000, scale_lo=6, scale_hi=16, ef_lo=4, ef_hi=32))
    if number == 5:
        g = GraphSpec("rmat", scale or 28, 16, seed, ("bursty", 64), ("uniform", 8))
        return Workload(5, "served-rmat-s%d" % g.scale, g, ("count", "close_hist", "label_table"), 8,
                        extra=dict(pool_scale_lo=16, pool_scale_hi=20))
    raise ValueError(number)


def batch_graph_spec(g: int, master: int = MASTER_SEED + 4, scale_lo: int = 6, scale_hi: int = 16,
                     ef_lo: int = 4, ef_hi: int = 32) -> GraphSpec:
    """Recipe of graph g of the batched workload: R-MAT or Erdos-Renyi 50/50,
    scale uniform in [scale_lo, scale_hi], edge factor uniform in
    [ef_lo, ef_hi], timestamps uniform on [0, 2^20), labels uniform 0..7."""
    lib = _load()
    sg = ctypes.c_uint64()
    kind = ctypes.c_uint32()
    sc = ctypes.c_uint32()
    ef = ctypes.c_uint32()
    lib.tpgen_batch_params(master, g, scale_lo, scale_hi, ef_lo, ef_hi,
                           ctypes.byref(sg), ctypes.byref(kind), ctypes.byref(sc), ctypes.byref(ef))
    return GraphSpec("er" if kind.value else "rmat", sc.value, ef.value, sg.value,
                     ("uniform", 20), ("uniform", 8))


def batch_specs(n_graphs: int, master: int = MASTER_SEED + 4, scale_lo: int = 6, scale_hi: int = 16,
                ef_lo: int = 4, ef_hi: int = 32) -> list:
    """Recipes of graphs 0..n_graphs-1 of a batch (see batch_graph_spec)."""
    return [batch_graph_spec(g, master, scale_lo, scale_hi, ef_lo, ef_hi) for g in range(n_graphs)]


def batch_offsets(specs: list) -> tuple:
    """(edge_offsets uint64[G+1], vertex_counts uint32[G]) of a batch."""
    eoff = np.zeros(len(specs) + 1, np.uint64)
    eoff[1:] = np.cumsum([s.n_edges for s in specs], dtype=np.uint64)
    vcnt = np.array([s.n for s in specs], np.uint32)
    return eoff, vcnt


def generate_batch(specs: list) -> dict:
    """Concatenated raw inputs of a batch: src, dst, ts (uint32, local ids),
    vlab (uint8), edge_offsets, vertex_counts."""
    eoff, vcnt = batch_offsets(specs)
    M, N = int(eoff[-1]), int(vcnt.sum())
    src = np.empty(M, np.uint32)
    dst = np.empty(M, np.uint32)
    ts = np.empty(M, np.uint32)
    vlab = np.empty(N, np.uint8)
    v0 = 0
    for i, s in enumerate(specs):
        e0, e1 = int(eoff[i]), int(eoff[i + 1])
        fill_edges(s, src[e0:e1], dst[e0:e1])
        fill_ts(s, ts[e0:e1])
        fill_labels(s, vlab[v0:v0 + s.n])
        v0 += s.n
    return dict(src=src, dst=dst, ts=ts, vlab=vlab, edge_offsets=eoff, vertex_counts=vcnt)


# --------------------------------------------------------------------------
# Device generation of a batch (tpgen_dev.hip): the same values as
# generate_batch, written straight into device memory.
# --------------------------------------------------------------------------

_dev_lib = None
_DEV_GRAPH = np.dtype([("seed", np.uint64), ("edge_offset", np.uint64), ("n_edges", np.uint64),
                       ("vertex_offset", np.uint64), ("kind", np.uint32), ("scale", np.uint32),
                       ("ts_bits", np.uint32), ("n_labels", np.uint32)])
_DEV_CHUNK = np.dtype([("graph", np.uint32), ("count", np.uint32), ("first", np.uint64)])
_CHUNK_EDGES = 1 << 16


def _load_dev():
    global _dev_lib
    if _dev_lib is not None:
        return _dev_lib
    if not os.path.exists(_DEV_LIB):
        raise ImportError("libtpgen_dev.so is not built (run synth.build())")
    lib = ctypes.CDLL(_DEV_LIB)
    p, u32 = ctypes.c_void_p, ctypes.c_uint32
    lib.tpgen_dev_batch.restype = ctypes.c_int
    lib.tpgen_dev_batch.argtypes = [p, u32, p, u32, u32, u32, u32, p, p, p, p, p]
    _dev_lib = lib
    return lib


def generate_batch_device(specs: list, torch, stream=None) -> dict:
    """Raw inputs of a batch of uniform-time, uniform-label graphs generated
    on the current device: int32 tensors src, dst, ts (uint32 values, local
    ids) and a uint8 tensor vlab, with host arrays edge_offsets and
    vertex_counts.  Byte for byte the arrays of generate_batch(specs)."""
    eoff, vcnt = batch_offsets(specs)
    G = len(specs)
    recs = np.zeros(G, _DEV_GRAPH)
    voff = 0
    chunks = []
    for i, s in enumerate(specs):
        if s.ts[0] != "uniform" or s.labels[0] != "uniform":
            raise ValueError("device batches take uniform times and labels")
        recs[i] = (s.seed, int(eoff[i]), s.n_edges, voff, 0 if s.kind == "rmat" else 1, s.scale, s.ts[1],
                   s.labels[1])
        voff += s.n
        nch = -(-s.n_edges // _CHUNK_EDGES)
        if nch:
            first = np.arange(nch, dtype=np.uint64) * _CHUNK_EDGES
            cnt = np.minimum(np.uint64(s.n_edges) - first, _CHUNK_EDGES).astype(np.uint32)
            ch = np.zeros(nch, _DEV_CHUNK)
            ch["graph"], ch["count"], ch["first"] = i, cnt, first
            chunks.append(ch)
    chunks = np.concatenate(chunks) if chunks else np.zeros(0, _DEV_CHUNK)
    M, N = int(eoff[-1]), int(vcnt.sum())
    dev = "cuda"
    d_recs = torch.from_numpy(recs.view(np.uint8)).to(dev)
    d_chunks = torch.from_numpy(chunks.view(np.uint8)).to(dev)
    src = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    ts = torch.empty_like(src)
    vlab = torch.empty(max(N, 1), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = _load_dev().tpgen_dev_batch(d_recs.data_ptr(), G, d_chunks.data_ptr(), len(chunks), *RMAT_THR,
                                     src.data_ptr(), dst.data_ptr(), ts.data_ptr(), vlab.data_ptr(), stream)
    if st != 0:
        raise RuntimeError("tpgen_dev_batch: hip error %d" % st)
    torch.cuda.synchronize()
    del d_recs, d_chunks
    return dict(src=src[:M], dst=dst[:M], ts=ts[:M], vlab=vlab[:N], edge_offsets=eoff, vertex_counts=vcnt)
