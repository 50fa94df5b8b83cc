// survey.hip -- the triangle survey on the degree-ordered directed graph.
//
// Algorithm 1 visits, for every edge p -> q, the rest of Adj+(p) after q
// (the candidate closing vertices r) and intersects it with Adj+(q).  The
// kernels here group that work by the target q (the vertex that receives the
// push in Algorithm 1): a workgroup loads Adj+^m(q) -- target ranks, edge
// times and target labels -- into an LDS hash table once, then streams the
// candidate rows of many pivots p and probes each candidate against the
// table.  Every probe is one wedge check; every hit is one triangle
// p <+ q <+ r with all six metadata items at hand:
//   meta(p) and meta(p,q)    from the in-edge record of p -> q
//   meta(p,r)                from p's row, next to the streamed candidate
//   meta(q)                  per tile
//   meta(q,r) and meta(r)    from the hash slot of r
// (the co-location argument of the Push-Only subsection).  Hits are reduced
// into LDS counters (the counting set of the Containers subsection, one per
// workgroup) that are merged into the result with global atomics when the
// workgroup retires.
//
// Work is a list of tiles (at most kTileRecords in-edge records of one q);
// persistent workgroups take tiles from an atomic counter.  Targets are
// split into three classes by d+(q): LDS hash of <= 2048 slots, LDS hash of
// <= 8192 slots, and binary search of Adj+(q) in HBM for the rest.
#include <algorithm>

#include "graph.hpp"
#include "plan.hpp"

using namespace tp;

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kUnroll = 8;
constexpr uint32_t kEmpty = 0xffffffffu;
constexpr uint32_t kHashMul = 0x9e3779b1u;  // Fibonacci hashing

struct SurveyParams {
    const uint64_t *rowptr;
    const uint32_t *col;
    const uint32_t *ets;
    const uint8_t *tlab;
    const uint8_t *rlab;
    const InRec *inrec;
    const TileDesc *tiles;
    uint64_t n_tiles;
    unsigned long long *tile_counter;
    unsigned long long *out;  // TP_RESULT_WORDS
    uint32_t outputs, filters;
    uint32_t table_words;     // entries of the label table in LDS (0 if unused)
    uint32_t oc_words;        // 1024 if OPEN_CLOSE else 0
    uint64_t spread_lt, t_lo, t_hi;
    uint64_t label_mask[13];
    // enumeration
    uint32_t *enum_out;
    uint64_t enum_cap;
    unsigned long long *enum_count;
    const uint32_t *perm;
    uint32_t n;
};

// LDS layout (dynamic): [hash keys][hash times][hash labels][record starts]
// [record prefix][record times][record labels][counters].
struct LdsLayout {
    uint32_t slots;
    size_t off_hts, off_hlab, off_rk, off_rpre, off_rts, off_rlab, off_cnt, total;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline LdsLayout lds_layout(uint32_t slots, bool meta, uint32_t counter_words)
{
    LdsLayout L;
    L.slots = slots;
    size_t o = (size_t)slots * 4;
    L.off_hts = o;
    if (meta) o += (size_t)slots * 4;
    L.off_hlab = o;
    if (meta) o += slots;
    o = align_up(o, 8);
    L.off_rk = o;
    o += (size_t)kTileRecords * 8;
    L.off_rpre = o;
    o += (size_t)(kTileRecords + 16) * 4;
    L.off_rts = o;
    if (meta) o += (size_t)kTileRecords * 4;
    L.off_rlab = o;
    if (meta) o += kTileRecords;
    o = align_up(o, 8);
    L.off_cnt = o;
    o += (size_t)counter_words * 8;
    L.total = o;
    return L;
}

// counters in LDS: [hist 32][table table_words][open_close oc_words]
__host__ __device__ inline uint32_t counter_words(uint32_t table_words, uint32_t oc_words)
{
    return 32 + table_words + oc_words;
}

__device__ __forceinline__ uint32_t close_bin(uint32_t d)
{
    // ceil(log2 d) for d >= 2 is the bit length of d - 1; d = 0, 1 -> 0; cap 31
    if (d <= 1) return 0;
    const uint32_t b = 32u - (uint32_t)__clz(d - 1);
    return b > 31 ? 31 : b;
}

__device__ __forceinline__ uint32_t multiset_index(uint32_t a, uint32_t b, uint32_t c)
{
    // sort three labels, then the colex rank C(c+2,3) + C(b+1,2) + a
    uint32_t lo = min(a, b), hi = max(a, b);
    uint32_t x = min(lo, c), z = max(hi, c);
    uint32_t y = a + b + c - x - z;
    return (z + 2) * (z + 1) * z / 6 + (y + 1) * y / 2 + x;
}

struct Hit {
    uint32_t t_pq, t_pr, t_qr;
    uint32_t l_p, l_q, l_r;
};

// Reduce one triangle into the workgroup's counters.  Returns 1 if it passed
// the filters.
__device__ __forceinline__ uint32_t reduce_hit(const SurveyParams &P, const Hit &h, unsigned long long *cnt,
                                               const uint64_t *mask_lds, unsigned long long &spread)
{
    const uint32_t f = P.filters;
    if (f & TP_FILT_WINDOW) {
        if (h.t_pq < P.t_lo || h.t_pq > P.t_hi || h.t_pr < P.t_lo || h.t_pr > P.t_hi || h.t_qr < P.t_lo ||
            h.t_qr > P.t_hi)
            return 0;
    }
    uint32_t idx = 0;
    if ((P.outputs & TP_OUT_LABEL_TABLE) || (f & TP_FILT_LABEL_MASK)) idx = multiset_index(h.l_p, h.l_q, h.l_r);
    if (f & TP_FILT_LABEL_MASK) {
        if (!((mask_lds[idx >> 6] >> (idx & 63)) & 1ull)) return 0;
    }
    const uint32_t t1 = min(min(h.t_pq, h.t_pr), h.t_qr);
    const uint32_t t3 = max(max(h.t_pq, h.t_pr), h.t_qr);
    const uint32_t close = t3 - t1;
    if (P.outputs & TP_OUT_CLOSE_HIST) atomicAdd(&cnt[close_bin(close)], 1ull);
    if (P.outputs & TP_OUT_LABEL_TABLE) atomicAdd(&cnt[32 + idx], 1ull);
    if (P.outputs & TP_OUT_SPREAD_COUNT) spread += ((uint64_t)close < P.spread_lt) ? 1ull : 0ull;
    if (P.outputs & TP_OUT_OPEN_CLOSE) {
        const uint32_t t2 = h.t_pq + h.t_pr + h.t_qr - t1 - t3;  // exact in uint32 arithmetic mod 2^32
        atomicAdd(&cnt[32 + P.table_words + close_bin(t2 - t1) * 32 + close_bin(close)], 1ull);
    }
    return 1;
}

// Binary search of r in col[lo, lo+len); returns the index or -1.
__device__ __forceinline__ int64_t global_find(const uint32_t *col, uint64_t lo, uint32_t len, uint32_t r)
{
    uint32_t a = 0, b = len;
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        const uint32_t v = col[lo + mid];
        if (v < r) a = mid + 1;
        else b = mid;
    }
    return (a < len && col[lo + a] == r) ? (int64_t)(lo + a) : -1;
}

__device__ __forceinline__ uint32_t find_pivot(const uint64_t *rowptr, uint32_t n, uint64_t k)
{
    // the row p with rowptr[p] <= k < rowptr[p+1]
    uint32_t a = 0, b = n;
    while (b - a > 1) {
        const uint32_t mid = a + (b - a) / 2;
        if (rowptr[mid] <= k) a = mid;
        else b = mid;
    }
    return a;
}

// LOG_SLOTS > 0: LDS hash of Adj+(q) with 2^LOG_SLOTS slots at most.
// LOG_SLOTS == 0: binary search of Adj+(q) in HBM.
template <int LOG_SLOTS, bool META, bool ENUM>
__global__ __launch_bounds__(kBlock) void survey_kernel(SurveyParams P)
{
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr uint32_t kSlots = LOG_SLOTS > 0 ? (1u << LOG_SLOTS) : 0u;
    const LdsLayout L = lds_layout(kSlots, META, counter_words(P.table_words, P.oc_words));
    uint32_t *hkey = reinterpret_cast<uint32_t *>(lds);
    uint32_t *hts = reinterpret_cast<uint32_t *>(lds + L.off_hts);
    uint8_t *hlab = lds + L.off_hlab;
    uint64_t *rk = reinterpret_cast<uint64_t *>(lds + L.off_rk);
    uint32_t *rpre = reinterpret_cast<uint32_t *>(lds + L.off_rpre);
    uint32_t *rts = reinterpret_cast<uint32_t *>(lds + L.off_rts);
    uint8_t *rlb = lds + L.off_rlab;
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(lds + L.off_cnt);
    __shared__ uint64_t mask_lds[13];
    __shared__ unsigned long long s_tile;
    __shared__ uint32_t s_scan[kWaves];

    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const uint32_t lane = lane_id();
    const uint32_t nc = counter_words(P.table_words, P.oc_words);
    for (uint32_t i = tid; i < nc; i += kBlock) cnt[i] = 0;
    if (tid < 13) mask_lds[tid] = P.label_mask[tid];

    unsigned long long my_tri = 0, my_spread = 0, probes = 0;

    for (;;) {
        if (tid == 0) s_tile = atomicAdd(P.tile_counter, 1ull);
        __syncthreads();
        const unsigned long long ti = s_tile;
        if (ti >= P.n_tiles) break;
        const TileDesc d = P.tiles[P.n_tiles - 1 - ti];
        const uint32_t q = d.q;
        const uint32_t nrec = d.cnt;
        const uint64_t kq = P.rowptr[q];
        const uint32_t dq = (uint32_t)(P.rowptr[q + 1] - kq);
        const uint32_t l_q = META ? P.rlab[q] : 0u;

        uint32_t log_s = 0, smask = 0;
        if (LOG_SLOTS > 0) {
            // slots: the power of two >= 2*dq, at least 64
            log_s = 6;
            while ((1u << log_s) < 2u * dq) ++log_s;
            smask = (1u << log_s) - 1;
            for (uint32_t i = tid; i <= smask; i += kBlock) hkey[i] = kEmpty;
        }
        // in-edge records of this tile, and the prefix of their lengths
        uint32_t lens[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t i = tid * 2 + j;
            lens[j] = 0;
            if (i < nrec) {
                const InRec r = P.inrec[d.e0 + i];
                const uint64_t k = (uint64_t)r.k_lo | ((uint64_t)(r.k_hi_lab & 0xffffffu) << 32);
                rk[i] = k + 1;  // first candidate slot
                lens[j] = r.len;
                if (META) {
                    rts[i] = r.t_pq;
                    rlb[i] = (uint8_t)(r.k_hi_lab >> 24);
                }
            }
        }
        uint32_t total;
        const uint32_t pre = block_excl_scan<kBlock>(lens[0] + lens[1], s_scan, total);
        if (tid * 2 < kTileRecords) {
            rpre[tid * 2] = pre;
            rpre[tid * 2 + 1] = pre + lens[0];
        }
        // records past the tile end: prefix = total (so that searches stop)
        __syncthreads();
        for (uint32_t i = nrec + tid; i < kTileRecords + 16; i += kBlock) rpre[i] = (i == nrec) ? total : 0xffffffffu;
        if (LOG_SLOTS > 0) {
            for (uint32_t i = tid; i < dq; i += kBlock) {
                const uint32_t r = P.col[kq + i];
                uint32_t h = (r * kHashMul) >> (32 - log_s);
                for (;;) {
                    const uint32_t prev = atomicCAS(&hkey[h], kEmpty, r);
                    if (prev == kEmpty) break;
                    h = (h + 1) & smask;
                }
                if (META) {
                    hts[h] = P.ets[kq + i];
                    hlab[h] = P.tlab[kq + i];
                }
            }
        }
        __syncthreads();
        if (tid == 0) probes += total;

        // ---- stream the candidates: wave w takes a contiguous range of rows
        const uint32_t rows = (total + kWave - 1) / kWave;
        const uint32_t row_lo = (uint32_t)((uint64_t)rows * w / kWaves);
        const uint32_t row_hi = (uint32_t)((uint64_t)rows * (w + 1) / kWaves);
        uint32_t seg = 0;
        for (uint32_t row = row_lo; row < row_hi; row += kUnroll) {
            uint64_t addr[kUnroll];
            uint32_t segj[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) {
                const uint32_t f = (row + j) * kWave + lane;
                ok[j] = (row + j < row_hi) && f < total;
                if (ok[j]) {
                    while (rpre[seg + 8] <= f) seg += 8;
                    while (rpre[seg + 1] <= f) ++seg;
                    addr[j] = rk[seg] + (f - rpre[seg]);
                    segj[j] = seg;
                }
            }
            uint32_t cand[kUnroll], tpr[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) {
                if (ok[j]) {
                    cand[j] = P.col[addr[j]];
                    if (META) tpr[j] = P.ets[addr[j]];
                }
            }
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) {
                if (!ok[j]) continue;
                const uint32_t r = cand[j];
                int64_t slot = -1;
                if (LOG_SLOTS > 0) {
                    uint32_t h = (r * kHashMul) >> (32 - log_s);
                    for (;;) {
                        const uint32_t key = hkey[h];
                        if (key == r) { slot = h; break; }
                        if (key == kEmpty) break;
                        h = (h + 1) & smask;
                    }
                } else {
                    slot = global_find(P.col, kq, dq, r);
                }
                if (slot < 0) continue;
                if (!META && !ENUM) {
                    ++my_tri;
                    continue;
                }
                Hit h;
                h.t_pq = rts[segj[j]];
                h.l_p = rlb[segj[j]];
                h.l_q = l_q;
                h.t_pr = tpr[j];
                if (LOG_SLOTS > 0) {
                    h.t_qr = hts[slot];
                    h.l_r = hlab[slot];
                } else {
                    h.t_qr = P.ets[slot];
                    h.l_r = P.tlab[slot];
                }
                if (ENUM) {
                    const unsigned long long at = atomicAdd(P.enum_count, 1ull);
                    if (at < P.enum_cap) {
                        const uint64_t kpq = rk[segj[j]] - 1;
                        const uint32_t p = find_pivot(P.rowptr, P.n, kpq);
                        uint32_t *o = P.enum_out + at * 9;
                        o[0] = P.perm[p];
                        o[1] = P.perm[q];
                        o[2] = P.perm[r];
                        o[3] = h.t_pq;
                        o[4] = h.t_pr;
                        o[5] = h.t_qr;
                        o[6] = h.l_p;
                        o[7] = h.l_q;
                        o[8] = h.l_r;
                    }
                    ++my_tri;
                } else {
                    my_tri += reduce_hit(P, h, cnt, mask_lds, my_spread);
                }
            }
        }
        __syncthreads();
    }

    // ---- merge this workgroup's counters into the result
    my_tri = wave_sum(my_tri);
    my_spread = wave_sum(my_spread);
    if (lane == 0) {
        if (my_tri) atomicAdd(&P.out[TP_RW_TRIANGLES], my_tri);
        if (my_spread) atomicAdd(&P.out[TP_RW_SPREAD], my_spread);
    }
    if (tid == 0 && probes) atomicAdd(&P.out[TP_RW_PROBES], probes);
    __syncthreads();
    for (uint32_t i = tid; i < nc; i += kBlock) {
        const unsigned long long v = cnt[i];
        if (!v) continue;
        uint32_t word;
        if (i < 32) word = TP_RW_HIST + i;
        else if (i < 32 + P.table_words) word = TP_RW_TABLE + (i - 32);
        else word = TP_RW_OPEN_CLOSE + (i - 32 - P.table_words);
        atomicAdd(&P.out[word], v);
    }
}

__global__ void zero_u64(unsigned long long *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

uint32_t table_size(uint32_t L) { return (L + 2) * (L + 1) * L / 6; }

template <int LOG_SLOTS, bool META, bool ENUM>
void launch_class(const SurveyParams &P, hipStream_t s, int device)
{
    if (P.n_tiles == 0) return;
    const uint32_t slots = LOG_SLOTS > 0 ? (1u << LOG_SLOTS) : 0u;
    const LdsLayout L = lds_layout(slots, META, counter_words(P.table_words, P.oc_words));
    auto kern = survey_kernel<LOG_SLOTS, META, ENUM>;
    TP_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total));
    int per_cu = 0;
    TP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, L.total));
    if (per_cu < 1) fail(TP_ERR_DEVICE, "survey kernel does not fit on a compute unit");
    int cus = 0;
    TP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    uint64_t grid = (uint64_t)per_cu * cus;
    if (grid > P.n_tiles) grid = P.n_tiles;
    zero_u64<<<1, 64, 0, s>>>(P.tile_counter, 1);
    TP_CHECK_LAUNCH();
    kern<<<(unsigned)grid, kBlock, L.total, s>>>(P);
    TP_CHECK_LAUNCH();
}

template <bool META, bool ENUM>
void launch_all(const tp_graph *g, SurveyParams P, uint32_t strategy, hipStream_t s)
{
    // one tile counter per class, so the three launches may overlap later
    if (strategy == TP_STRAT_GLOBAL_SEARCH) {
        for (int c = 0; c < kNumClasses; ++c) {
            P.tiles = g->tiles[c].get();
            P.n_tiles = g->n_tiles[c];
            launch_class<0, META, ENUM>(P, s, g->device);
        }
        return;
    }
    P.tiles = g->tiles[kClassSmall].get();
    P.n_tiles = g->n_tiles[kClassSmall];
    launch_class<kSmallLogSlots, META, ENUM>(P, s, g->device);
    P.tiles = g->tiles[kClassLarge].get();
    P.n_tiles = g->n_tiles[kClassLarge];
    launch_class<kLargeLogSlots, META, ENUM>(P, s, g->device);
    P.tiles = g->tiles[kClassHuge].get();
    P.n_tiles = g->n_tiles[kClassHuge];
    launch_class<0, META, ENUM>(P, s, g->device);
}

void validate_spec(const tp_graph *g, const tp_survey_spec *sp)
{
    if (!g || !sp) fail(TP_ERR_INVALID, "tripoll_survey: NULL argument");
    const uint32_t known = TP_OUT_COUNT | TP_OUT_CLOSE_HIST | TP_OUT_LABEL_TABLE | TP_OUT_SPREAD_COUNT |
                           TP_OUT_OPEN_CLOSE;
    if (sp->outputs & ~known) fail(TP_ERR_INVALID, "tripoll_survey: unknown output bits");
    if (sp->filters & ~(TP_FILT_WINDOW | TP_FILT_LABEL_MASK)) fail(TP_ERR_INVALID, "tripoll_survey: unknown filter bits");
    if (sp->strategy > TP_STRAT_GLOBAL_SEARCH) fail(TP_ERR_INVALID, "tripoll_survey: unknown strategy");
    const bool labels = (sp->outputs & TP_OUT_LABEL_TABLE) || (sp->filters & TP_FILT_LABEL_MASK);
    if (labels) {
        if (sp->n_labels < 1 || sp->n_labels > TP_MAX_LABELS)
            fail(TP_ERR_INVALID, "tripoll_survey: n_labels must be in 1..16");
        if (g->stats.max_label >= sp->n_labels)
            fail(TP_ERR_INVALID, "tripoll_survey: graph has label " + std::to_string(g->stats.max_label) +
                                     " >= n_labels " + std::to_string(sp->n_labels));
    }
    if ((sp->filters & TP_FILT_WINDOW) && sp->t_lo > sp->t_hi)
        fail(TP_ERR_INVALID, "tripoll_survey: t_lo > t_hi");
}

SurveyParams make_params(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *out,
                         unsigned long long *counter)
{
    SurveyParams P{};
    P.rowptr = g->rowptr.get();
    P.col = g->col.get();
    P.ets = g->ets.get();
    P.tlab = g->tlab.get();
    P.rlab = g->rlab.get();
    P.inrec = g->inrec.get();
    P.tile_counter = counter;
    P.out = out;
    P.outputs = sp->outputs | TP_OUT_COUNT;
    P.filters = sp->filters;
    P.table_words = (sp->outputs & TP_OUT_LABEL_TABLE) ? table_size(sp->n_labels) : 0;
    P.oc_words = (sp->outputs & TP_OUT_OPEN_CLOSE) ? 1024 : 0;
    P.spread_lt = sp->spread_lt;
    P.t_lo = sp->t_lo;
    P.t_hi = sp->t_hi;
    // window bounds beyond the uint32 time range clamp to it
    if (P.t_hi > 0xffffffffull) P.t_hi = 0xffffffffull;
    for (int i = 0; i < 13; ++i) P.label_mask[i] = sp->label_mask[i];
    P.perm = g->perm.get();
    P.n = g->n;
    return P;
}

bool needs_meta(const tp_survey_spec *sp)
{
    return (sp->outputs & ~TP_OUT_COUNT) != 0 || sp->filters != 0;
}

// Enqueue a whole survey into the caller's result buffer (which also holds
// the tile counter).  Allocates nothing.
template <bool ENUM>
void survey_enqueue(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *dev_out, hipStream_t s,
                    uint32_t *enum_out = nullptr, uint64_t enum_cap = 0)
{
    zero_u64<<<grid_for(TP_RESULT_WORDS, 256), 256, 0, s>>>(dev_out, TP_RESULT_WORDS);
    TP_CHECK_LAUNCH();
    SurveyParams P = make_params(g, sp, dev_out, dev_out + TP_RW_SCRATCH);
    if (g->m == 0 || g->n_in == 0) return;
    if (ENUM) {
        P.enum_out = enum_out;
        P.enum_cap = enum_cap;
        P.enum_count = dev_out + TP_RW_SCRATCH + 1;
        launch_all<true, true>(g, P, TP_STRAT_AUTO, s);
    } else if (needs_meta(sp)) {
        launch_all<true, false>(g, P, sp->strategy, s);
    } else {
        launch_all<false, false>(g, P, sp->strategy, s);
    }
}

void copy_result(const std::vector<unsigned long long> &h, tp_survey_result *out)
{
    std::memset(out, 0, sizeof(*out));
    out->triangles = h[TP_RW_TRIANGLES];
    out->spread_count = h[TP_RW_SPREAD];
    out->probes = h[TP_RW_PROBES];
    for (int i = 0; i < 32; ++i) out->close_hist[i] = h[TP_RW_HIST + i];
    for (uint32_t i = 0; i < TP_TABLE_MAX; ++i) out->label_table[i] = h[TP_RW_TABLE + i];
    for (int i = 0; i < 1024; ++i) out->open_close[i] = h[TP_RW_OPEN_CLOSE + i];
}

}  // namespace

// ================================================================ C ABI

extern "C" tp_status tripoll_survey(const tp_graph *g, const tp_survey_spec *spec, tp_survey_result *out, void *stream)
{
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_survey: NULL result");
        validate_spec(g, spec);
        hipStream_t s = (hipStream_t)stream;
        DArray<unsigned long long> res(TP_RESULT_WORDS, s);
        EventTimer all(s), kern(s);
        all.start();
        kern.start();
        survey_enqueue<false>(g, spec, res.get(), s);
        kern.stop();
        std::vector<unsigned long long> h(TP_RESULT_WORDS);
        TP_HIP(hipMemcpyAsync(h.data(), res.get(), TP_RESULT_WORDS * 8, hipMemcpyDeviceToHost, s));
        all.stop();
        TP_HIP(hipStreamSynchronize(s));
        copy_result(h, out);
        out->kernel_ms = kern.ms();
        out->total_ms = all.ms();
    });
}

extern "C" tp_status tripoll_survey_async(const tp_graph *g, const tp_survey_spec *spec, uint64_t *dev_out,
                                          void *stream)
{
    return guard([&] {
        if (!dev_out) fail(TP_ERR_INVALID, "tripoll_survey_async: NULL output");
        validate_spec(g, spec);
        survey_enqueue<false>(g, spec, reinterpret_cast<unsigned long long *>(dev_out), (hipStream_t)stream);
    });
}

extern "C" tp_status tripoll_enumerate(const tp_graph *g, uint32_t *dev_records, uint64_t capacity,
                                       uint64_t *n_found, void *stream)
{
    return guard([&] {
        if (!g || !n_found || (capacity && !dev_records)) fail(TP_ERR_INVALID, "tripoll_enumerate: bad argument");
        hipStream_t s = (hipStream_t)stream;
        tp_survey_spec sp{};
        sp.outputs = TP_OUT_COUNT;
        DArray<unsigned long long> res(TP_RESULT_WORDS, s);
        survey_enqueue<true>(g, &sp, res.get(), s, dev_records, capacity);
        unsigned long long found = 0;
        TP_HIP(hipMemcpyAsync(&found, res.get() + TP_RW_TRIANGLES, 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        *n_found = found;
    });
}
