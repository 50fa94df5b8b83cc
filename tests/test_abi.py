"""The C-ABI library loads, exports every declared entry point, and the
binding's structs match the header's layout (CPU only: no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2107_12330_amd import tripoll as tp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for f in os.listdir(INCLUDE):
        if f.endswith(".h"):
            text = open(os.path.join(INCLUDE, f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(tripoll_\w+)\s*\(", text, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = tp.load()
    names = declared_functions()
    assert "tripoll_build" in names and "tripoll_survey" in names
    for name in sorted(names):
        assert hasattr(lib, name), name
    # and the binding covers them all
    assert names <= set(tp.SIGNATURES)


def test_nm_lists_symbols():
    out = subprocess.check_output(["nm", "-D", "--defined-only", tp.LIB_PATH]).decode()
    exported = set(re.findall(r" T (tripoll_\w+)", out))
    assert declared_functions() <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "tripoll.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(tp_edge_list), sizeof(tp_graph_stats), sizeof(tp_survey_spec),
         sizeof(tp_survey_result));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(tp_graph_stats, phase_ms), offsetof(tp_survey_spec, label_mask),
         offsetof(tp_survey_result, kernel_ms), offsetof(tp_graph_stats, class_probes),
         offsetof(tp_survey_result, class_ms));
  printf("%u %u %u %u %u %u\\n", TP_RW_TABLE, TP_RW_OPEN_CLOSE, TP_RW_SCRATCH, TP_RESULT_WORDS, TP_RW_MAX_EDGE,
         TP_RW_DEGREE);
  printf("%zu %zu %zu %zu %u\\n", offsetof(tp_survey_spec, max_edge_shift), offsetof(tp_survey_result, max_edge),
         offsetof(tp_survey_result, degree_table), offsetof(tp_survey_result, directed), TP_RW_DIRECTED);
  printf("%zu %zu %zu %zu %u %u %u\\n", sizeof(tp_batch_edges), sizeof(tp_plan), sizeof(tp_tune_result),
         offsetof(tp_tune_result, trials), TP_BW_TABLE, TP_BATCH_SCRATCH_WORDS, TP_NUM_CLASSES);
  printf("%zu %zu %zu %zu %zu\\n", sizeof(tp_server_config), sizeof(tp_request_info), sizeof(tp_server_stats),
         offsetof(tp_server_stats, p50_ms), offsetof(tp_server_stats, elapsed_s));
  printf("%zu %u %u\\n", offsetof(tp_survey_result, class_triangles), TP_RW_CLASS_TRI, TP_RW_SCRATCH_WORDS);
  return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", INCLUDE, str(src), "-o", str(exe)])
    l1, l2, l3, l3b, l4, l5, l6 = subprocess.check_output([str(exe)]).decode().split("\n")[:7]
    assert list(map(int, l1.split())) == [ctypes.sizeof(tp.tp_edge_list), ctypes.sizeof(tp.tp_graph_stats),
                                          ctypes.sizeof(tp.tp_survey_spec), ctypes.sizeof(tp.tp_survey_result)]
    assert list(map(int, l2.split())) == [tp.tp_graph_stats.phase_ms.offset, tp.tp_survey_spec.label_mask.offset,
                                          tp.tp_survey_result.kernel_ms.offset, tp.tp_graph_stats.class_probes.offset,
                                          tp.tp_survey_result.class_ms.offset]
    assert list(map(int, l3.split())) == [tp.TP_RW_TABLE, tp.TP_RW_OPEN_CLOSE, tp.TP_RW_SCRATCH,
                                          tp.TP_RESULT_WORDS, tp.TP_RW_MAX_EDGE, tp.TP_RW_DEGREE]
    assert list(map(int, l3b.split())) == [tp.tp_survey_spec.max_edge_shift.offset, tp.tp_survey_result.max_edge.offset,
                                           tp.tp_survey_result.degree_table.offset,
                                           tp.tp_survey_result.directed.offset, tp.TP_RW_DIRECTED]
    assert list(map(int, l4.split())) == [ctypes.sizeof(tp.tp_batch_edges), ctypes.sizeof(tp.tp_plan),
                                          ctypes.sizeof(tp.tp_tune_result), tp.tp_tune_result.trials.offset,
                                          tp.TP_BW_TABLE, tp.TP_BATCH_SCRATCH_WORDS, tp.TP_NUM_CLASSES]
    assert list(map(int, l5.split())) == [ctypes.sizeof(tp.tp_server_config), ctypes.sizeof(tp.tp_request_info),
                                          ctypes.sizeof(tp.tp_server_stats), tp.tp_server_stats.p50_ms.offset,
                                          tp.tp_server_stats.elapsed_s.offset]
    assert list(map(int, l6.split())) == [tp.tp_survey_result.class_triangles.offset, tp.TP_RW_CLASS_TRI,
                                          tp.TP_RESULT_WORDS - tp.TP_RW_SCRATCH]


def test_msidx_is_colex_rank():
    # host-side helper of the library; the multiset order is the colex order
    from itertools import combinations_with_replacement
    ms = sorted(combinations_with_replacement(range(16), 3), key=lambda x: (x[2], x[1], x[0]))
    for i, m in enumerate(ms):
        assert tp.tripoll_msidx(*m) == i
        assert tp.tripoll_msidx(m[2], m[0], m[1]) == i


def test_version_and_error_string():
    assert "gfx950" in tp.tripoll_version()
    assert isinstance(tp.load().tripoll_last_error(), bytes)


def test_null_arguments_rejected_without_gpu():
    # argument checks happen before any HIP call
    lib = tp.load()
    assert lib.tripoll_graph_stats(None, None) == tp.TP_ERR_INVALID
    assert b"NULL" in lib.tripoll_last_error()
    assert lib.tripoll_build(None, None, None) == tp.TP_ERR_INVALID
    assert lib.tripoll_survey(None, None, None, None) == tp.TP_ERR_INVALID


def test_product_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2107_12330_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
