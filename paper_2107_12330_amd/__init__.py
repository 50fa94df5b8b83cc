"""MI355X-native metadata triangle survey (TriPoll's hot path).

The product is ``libtripoll.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/tripoll.h``); ``tripoll`` is its ctypes binding.
"""
from . import tripoll  # noqa: F401
from .tripoll import (Graph, build_graph, edge_list, export, make_spec, result_dict,  # noqa: F401
                      survey, words_dict)
