// capi.hip -- C ABI entry points for graph handles and utilities.
#include <memory>

#include "graph.hpp"

namespace tp {
const char *last_error_cstr();
}

using namespace tp;

extern "C" tp_status tripoll_graph_stats(const tp_graph *g, tp_graph_stats *out)
{
    return guard([&] {
        if (!g || !out) fail(TP_ERR_INVALID, "tripoll_graph_stats: NULL argument");
        *out = g->stats;
    });
}

extern "C" tp_status tripoll_graph_free(tp_graph *g)
{
    return guard([&] {
        if (!g) return;
        int cur = 0;
        TP_HIP(hipGetDevice(&cur));
        if (cur != g->device) TP_HIP(hipSetDevice(g->device));
        delete g;
        if (cur != g->device) TP_HIP(hipSetDevice(cur));
    });
}

extern "C" tp_status tripoll_graph_export(const tp_graph *g, uint64_t *rowptr, uint32_t *col, uint32_t *etime,
                                          uint8_t *tlabel, uint32_t *rank_to_id, uint8_t *rank_label)
{
    return guard([&] {
        if (!g) fail(TP_ERR_INVALID, "tripoll_graph_export: NULL graph");
        const size_t n = g->n, m = g->m;
        if (rowptr) TP_HIP(hipMemcpy(rowptr, g->rowptr.get(), (n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
        if (col && m) TP_HIP(hipMemcpy(col, g->col.get(), m * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (etime && m) TP_HIP(hipMemcpy(etime, g->ets.get(), m * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (tlabel && m) TP_HIP(hipMemcpy(tlabel, g->tlab.get(), m, hipMemcpyDeviceToHost));
        if (rank_to_id) TP_HIP(hipMemcpy(rank_to_id, g->perm.get(), n * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (rank_label) TP_HIP(hipMemcpy(rank_label, g->rlab.get(), n, hipMemcpyDeviceToHost));
    });
}

extern "C" uint32_t tripoll_msidx(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t x = a < b ? a : b, z = a < b ? b : a;
    if (c < x) x = c;
    if (c > z) z = c;
    const uint32_t y = a + b + c - x - z;
    return (z + 2) * (z + 1) * z / 6 + (y + 1) * y / 2 + x;
}

extern "C" const char *tripoll_last_error(void) { return last_error_cstr(); }

extern "C" const char *tripoll_version(void) { return "tripoll-mi355x 0.1 (gfx950)"; }

extern "C" tp_status tripoll_trim(void)
{
    return guard([&] { dev_trim(); });
}

extern "C" tp_status tripoll_cached_bytes(uint64_t *out)
{
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_cached_bytes: NULL");
        *out = dev_cached_bytes();
    });
}

extern "C" tp_status tripoll_live_bytes(uint64_t *out)
{
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_live_bytes: NULL");
        *out = dev_live_bytes();
    });
}

extern "C" tp_status tripoll_fail_alloc_after(uint64_t n)
{
    return guard([&] { dev_fail_after(n); });
}
