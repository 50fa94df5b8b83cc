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
// Work is a list of tiles (a capped number of in-edge records of one q);
// persistent workgroups, or in the per-wave form single waves, take tiles
// from an atomic counter.  Targets are split into four classes by d+(q), and
// each class runs one variant of the kernel (the survey plan): LDS tables
// per wave for tiny targets, LDS tables per workgroup of <= 2 x 1024 or
// <= 2 x 4096 slots for small and large ones, and for huge ones the large
// tables again, one piece of Adj+(q) at a time (plan.hpp), over in-edge
// records cut to each piece's candidates by the planner; any class may be
// switched to binary search of Adj+(q) in HBM.
#include <algorithm>
#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>

#include "graph.hpp"
#include "multi.hpp"
#include "plan.hpp"

using namespace tp;

namespace {

constexpr int kSmallBlock = 256;   // 4 waves share a small target's tables
constexpr int kLargeBlock = 1024;  // 16 waves share a large target's tables
// Candidate loads in flight per wave: a chunk is kSub sub-rows of 64
// candidates of one record, a batch is kBatch chunks, and two batches are in
// flight.  The per-wave form serves short rows (tiny targets, small graphs;
// on the scale-26 workload 13.5 candidates per record): chunks of one
// sub-row, two of them per batch (2 sub-rows per chunk: 20,000-graph batch
// survey 572.6 against 540.0 ms).
template <bool WAVE> struct Depth {
    static constexpr int kSub = WAVE ? 1 : 4;
    static constexpr int kBatch = WAVE ? 2 : 1;
    static constexpr uint32_t kChunkCand = kSub * 64;
};
constexpr uint32_t kRing = 128;    // per-wave ring of queued hits: slot|label(p), time(p,r), time(p,q), p
// Tiles claimed with one atomic on the tile counter: at most 8 by a workgroup
// and 16 by a wave of the per-wave form, fewer when the class has too few
// tiles for every claimer to make about 8 claims (the tail stays balanced).
// Every claim is an atomic on one counter, which at 131 M tiny tiles (the
// 20,000-graph batch) serialises: 8 per wave took that batch's survey to
// 515 ms, 16 per wave and 8 per workgroup to about 450 ms.
constexpr uint32_t kMaxClaimGroup = 8;
constexpr uint32_t kMaxClaimWave = 16;
// The tiles of a batch's launch are cut into kClaimSegs contiguous segments,
// one per XCD, each with its own claim counter.  Workgroups are dispatched to
// the 8 XCDs round robin, so workgroup b starts on segment b % 8: the waves of
// one XCD then work through one stretch of graphs, whose rows its L2 holds,
// instead of every XCD fetching the same rows into its own L2 (20,000-graph
// batch: 1.87 -> 1.08 TB fetched by the survey).  A workgroup whose segment is
// used up takes what is left of the next ones.  A single graph keeps one
// counter: there all XCDs share one stretch of ranks, whose rows the
// device-wide last-level cache then holds once (scale 26: tiny class 8 ms
// with one counter, 14 ms with eight).
constexpr uint32_t kClaimSegs = 8;
static_assert(kClaimSegs <= kClaimWords && kClaimSegs == 8, "one claim counter per segment, 2^3 segments");
constexpr int kRsrcWord3 = 0x00020000;  // buffer resource word 3 for raw 32-bit loads on CDNA
constexpr uint32_t kEmpty = 0xffffffffu;
// kernel forms (see survey_kernel)
constexpr int kFormSurvey = 0;
constexpr int kFormExt = 1;
constexpr int kFormPart = 2;
// The plain metadata survey of the 1024-thread workgroup (large and huge
// targets, 16 waves per compute unit) keeps twice the ring and reduces its
// hits two to a lane, 128 at a time, so that the two hits' LDS reads and
// counter adds overlap (scale-26 large class 327.6 -> 319.5 ms), wherever
// the outputs' counters leave LDS for it (WIDE; not with the open/close
// histogram and a label table over many labels); the other kernels keep
// kRing and reduce 64 at a time.
template <bool WAVE, int BLOCK, bool META, bool ENUM, bool MULTI, int FORM, bool WIDE = true>
constexpr uint32_t ring_size()
{
    return (WIDE && !WAVE && BLOCK == 1024 && META && !ENUM && !MULTI && FORM == kFormSurvey) ? 2 * kRing : kRing;
}
// a drain leaves at most 127 queued; two sub-rows add at most 128 (the
// doubled ring), one sub-row at most 64 (kRing)
static_assert(2 * kRing >= (2 * kWave - 1) + 2 * kWave && kRing >= (kWave - 1) + kWave, "hit ring capacity");
constexpr uint32_t kMaxKicks = 64;  // cuckoo displacements before a key goes to the stash

// The two cuckoo hash functions, each onto 2^log_s slots: the low bits of
// the rank, and a multiplicative hash of the rank folded to 24 bits (a
// full-rate 24-bit multiply; a 32-bit multiply issues at a quarter of the
// rate).  Ranks are dense, so the low bits spread the out-neighbours of a
// target well; keys that collide in both tables go to the stash, and a
// target whose stash overflows is searched in HBM, so the hash quality
// affects only speed.
__device__ __forceinline__ uint32_t hash0(uint32_t r, uint32_t log_s) { return r & ((1u << log_s) - 1u); }
__device__ __forceinline__ uint32_t hash1(uint32_t r, uint32_t log_s)
{
    return (uint32_t)__umul24(r ^ (r >> 12), 0x9e3779u) >> (32 - log_s);
}

struct SurveyParams {
    const uint64_t *rowptr;
    const uint32_t *col;
    const uint32_t *ets;
    const uint8_t *tlab;
    const uint8_t *rlab;
    const uint64_t *inkey;    // sorted in-edge keys (q << kbits) | k
    const uint32_t *inpay;    // rest of the pivot's row | label(pivot) << 24
    // the records of the huge class's tiles, one per (record, piece) with
    // candidates in the piece: key ((q + skip) << kbits) | k (skip: the
    // candidates of the rest of p's row below the piece's ranks), payload as
    // inpay with the candidates in the piece; inkey and inpay for that
    // class's launches
    const uint64_t *piece_key;
    const uint32_t *piece_pay;
    uint32_t kbits;
    const TileDesc *tiles;
    uint64_t n_tiles;
    unsigned long long *tile_counter;  // kClaimSegs claim counters
    unsigned long long *out;  // result words (one block per graph of a batch)
    const uint32_t *rank_gid; // graph of each rank (batches), or null
    uint32_t g_stride;        // words per graph block
    uint32_t o_tri, o_spread, o_probes, o_hist, o_table, o_oc, o_maxe, o_deg;  // word offsets in a block
    uint32_t outputs, filters;
    uint32_t table_words;     // entries of the label table in LDS (0 if unused)
    uint32_t oc_words;        // 1024 if OPEN_CLOSE else 0
    uint32_t maxe_words;      // 1024 if MAX_EDGE else 0
    uint32_t deg_words;       // entries of the degree table in LDS (0 if unused)
    uint32_t max_edge_shift;  // MAX_EDGE bin width 2^max_edge_shift
    uint32_t copies;          // copies of the histogram and table counters (1, 2 or 4)
    uint32_t dir_words;       // 8 if DIRECTED else 0
    uint32_t o_dir;
    const uint8_t *edir;      // directions of the oriented edges (directed builds)
    uint8_t dir_type[64];     // triangle type by dir(p,q) << 4 | dir(p,r) << 2 | dir(q,r); 7 for none
    unsigned long long *part_edge;  // participation: one counter per CSR slot
    const uint32_t *dbin_rank;  // [32 per graph] first rank of degree bin >= k (DEGREE_TABLE)
    const uint64_t *dbin_slot;  // [32 per graph] first CSR slot of a rank of degree bin >= k
    uint32_t t_lo32, t_hi32;  // window, clamped to the uint32 time range
    uint32_t spread_le;       // spread counter: close <= spread_le ...
    uint32_t spread_any;      // ... and spread_lt > 0
    uint32_t window_empty;    // window lies above every uint32 time
    uint32_t lut_shift;       // labels < 2^lut_shift index the multiset table (0 if unused)
    uint32_t max_kicks;       // cuckoo displacements per key before the stash
    uint64_t label_mask[13];
    // enumeration: records go to enum_out[enum_count++] (at most enum_cap),
    // or, streaming, tile t's records to enum_out[tile_base[t] - chunk_base +
    // tile_cursor[t]++]; with tile_count set, records are only counted per tile
    uint32_t *enum_out;
    uint64_t enum_cap;
    unsigned long long *enum_count;
    const uint32_t *enum_srow;  // row (pivot rank) of every CSR slot
    const uint64_t *enum_tile_base;
    unsigned *enum_tile_cursor;
    unsigned *enum_tile_count;
    uint64_t enum_chunk_base;
    uint64_t tile_gbase;      // index of tiles[0] among all tiles of the graph
    const uint32_t *perm;
    uint32_t n;
    // multi-request passes: per slot a result block of slot_words words
    // (layout of a batch block) at out + slot * g_stride
    const SlotSpec *slots;
    uint32_t n_slots, slot_words, slot_labels;
    uint32_t grid_eighths;    // share of the device the persistent grid may fill (0 or 8: all)
    uint32_t claim;           // tiles a wave (per-wave form) or workgroup claims at a time
    uint32_t claim_seg_log;   // log2 of the claim segments (0 or 3)
    // exact counting set of Algorithm 3 (extended form): an open-addressing
    // table of maxe_mask + 1 slots; key value + 1 (0: empty) and its count
    unsigned long long *maxe_keys;
    unsigned long long *maxe_counts;
    uint64_t maxe_mask;
    unsigned *maxe_overflow;  // set when a value finds no slot
    // single-graph surveys: after class c, the running triangle count is
    // copied to class_tri[c] (so that each class's triangles are known)
    unsigned long long *class_tri;
};

// LDS layout (dynamic): [hash keys][hash times][hash labels]
// [row positions][slot counts][hit rings][counters][label lut].  Positions
// and slot counts exist in the participation form only, which has no rings.
struct LdsLayout {
    uint32_t slots;
    size_t off_hts, off_hlab, off_hdir, off_hbin, off_hpos, off_hcnt, off_ring, off_cnt, off_lut, total;
};
// (the enumeration form keeps each key's original id where participation
// keeps row positions)

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// bins: the degree bin of each key (extended form with the degree table)
__host__ __device__ inline LdsLayout lds_layout(uint32_t slots, bool meta, uint32_t counter_words, int waves,
                                                uint32_t lut_shift, bool part = false, bool dir = false,
                                                bool ids = false, bool bins = false, uint32_t ring = kRing)
{
    LdsLayout L;
    L.slots = slots;
    size_t o = (size_t)slots * 4;
    L.off_hts = o;
    if (meta) o += (size_t)slots * 4;
    L.off_hlab = o;
    if (meta) o += slots;
    L.off_hdir = o;
    if (dir) o += slots;
    L.off_hbin = o;
    if (bins) o += slots;
    o = align_up(o, 16);
    L.off_hpos = o;
    if (part || ids) o += (size_t)slots * 4;
    L.off_hcnt = o;
    if (part) o += (size_t)slots * 4;
    L.off_ring = o;
    if (meta && !part) o += (size_t)waves * ring * 16;
    L.off_cnt = o;
    o += (size_t)counter_words * 8;
    L.off_lut = o;
    if (meta) o += (size_t)2 << (3 * lut_shift);
    L.total = o;
    return L;
}

// Counters of a workgroup: [close hist 32][label table][open/close]
// [max-edge bins][degree table][directed types]; the last three in the
// extended form only.  The histogram and the table, which most hits update,
// are held in P.copies interleaved copies (bin b, copy c at b * copies + c;
// lane l adds to copy l % copies), so that the lanes of a wave that hit the
// same bin spread over several LDS addresses (4 copies: scale-26 survey
// 485 -> 444 ms).  The host takes 4, 2 or 1 copies, whichever fits LDS, and
// 8 for the 1024-thread kernels where 8 fit beside the doubled hit ring
// (scale-26 large class 311.4 -> 308.8 ms).  A multi-request pass holds one
// batch-layout block per request slot.
constexpr uint32_t kMaxCopies = 4;
constexpr uint32_t kMaxCopiesLarge = 8;

struct CounterBase {
    uint32_t table, oc, maxe, deg, dir, total;
};

__host__ __device__ inline CounterBase counter_base(const SurveyParams &P, bool ext)
{
    CounterBase b;
    b.table = 32 * P.copies;
    b.oc = b.table + P.table_words * P.copies;
    b.maxe = b.oc + P.oc_words;
    b.deg = b.maxe + (ext ? P.maxe_words : 0u);
    b.dir = b.deg + (ext ? P.deg_words : 0u);
    b.total = b.dir + (ext ? P.dir_words : 0u);
    return b;
}

template <bool MULTI, int FORM>
__host__ __device__ inline uint32_t counter_words(const SurveyParams &P)
{
    if (MULTI) return P.n_slots * P.slot_words;
    return counter_base(P, FORM == kFormExt).total;
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
    uint32_t b_p, b_q, b_r;  // degree bins (DEGREE_TABLE only)
    uint32_t dtype;          // directed type (DIRECTED only)
};

// Reduce one triangle into the workgroup's counters.  Returns 1 if it passed
// the filters.  `lut` maps the labels (a, b, c), packed in lut_shift-bit
// fields, to the label-multiset index.
// The prefilters alone: the window on the three times and the label-mask
// bit of the multiset (labels must be below 2^lut_shift when it is used).
// ARITH: the multiset index is computed rather than looked up in `lut`
// (the per-wave form, whose register budget a lookup's address and wait
// strain: 20,000-graph batch survey 466 -> 437 ms; the workgroup forms keep
// the lookup, which is faster there).
template <bool ARITH = false>
__device__ __forceinline__ uint32_t label_index(const SurveyParams &P, const Hit &h, const uint16_t *lut)
{
    if (ARITH) return multiset_index(h.l_p, h.l_q, h.l_r);
    return lut[(((h.l_p << P.lut_shift) | h.l_q) << P.lut_shift) | h.l_r];
}

template <bool ARITH = false>
__device__ __forceinline__ bool passes_filters(const SurveyParams &P, const Hit &h, const uint64_t *mask_lds,
                                               const uint16_t *lut)
{
    const uint32_t f = P.filters;
    if (f & TP_FILT_WINDOW) {
        if (P.window_empty) return false;
        if (h.t_pq < P.t_lo32 || h.t_pq > P.t_hi32 || h.t_pr < P.t_lo32 || h.t_pr > P.t_hi32 ||
            h.t_qr < P.t_lo32 || h.t_qr > P.t_hi32)
            return false;
    }
    if (f & TP_FILT_LABEL_MASK) {
        const uint32_t idx = label_index<ARITH>(P, h, lut);
        if (!((mask_lds[idx >> 6] >> (idx & 63)) & 1ull)) return false;
    }
    return true;
}

// One more triangle whose largest edge time is v, in the exact counting set:
// linear probing from a hash of v (the "lowbias32" integer mixer published
// with C. Wellons' hash-prospector); a slot, once claimed by a compare
// and swap, keeps its value, so a plain read that already shows v (or any
// other value) is final and only an empty-looking slot needs the atomic.
__device__ __forceinline__ void maxe_count(const SurveyParams &P, uint32_t v)
{
    const unsigned long long key = (unsigned long long)v + 1ull;
    uint32_t x = v;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    uint64_t s = x & P.maxe_mask;
    for (uint64_t probe = 0; probe <= P.maxe_mask; ++probe) {
        unsigned long long k = __hip_atomic_load(P.maxe_keys + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == 0ull) k = atomicCAS(P.maxe_keys + s, 0ull, key);
        if (k == 0ull || k == key) {
            atomicAdd(P.maxe_counts + s, 1ull);
            return;
        }
        s = (s + 1) & P.maxe_mask;
    }
    atomicOr(P.maxe_overflow, 1u);
}

template <bool EXT, bool ARITH = false>
__device__ __forceinline__ uint32_t reduce_hit(const SurveyParams &P, const Hit &h, unsigned long long *cnt,
                                               const uint64_t *mask_lds, const uint16_t *lut, uint32_t &spread)
{
    const uint32_t f = P.filters;
    if (f & TP_FILT_WINDOW) {
        if (P.window_empty) return 0;
        if (h.t_pq < P.t_lo32 || h.t_pq > P.t_hi32 || h.t_pr < P.t_lo32 || h.t_pr > P.t_hi32 ||
            h.t_qr < P.t_lo32 || h.t_qr > P.t_hi32)
            return 0;
    }
    uint32_t idx = 0;
    if ((P.outputs & TP_OUT_LABEL_TABLE) || (f & TP_FILT_LABEL_MASK))
        idx = label_index<ARITH>(P, h, lut);
    if (f & TP_FILT_LABEL_MASK) {
        if (!((mask_lds[idx >> 6] >> (idx & 63)) & 1ull)) return 0;
    }
    const uint32_t t1 = min(min(h.t_pq, h.t_pr), h.t_qr);
    const uint32_t t3 = max(max(h.t_pq, h.t_pr), h.t_qr);
    const uint32_t close = t3 - t1;
    const CounterBase B = counter_base(P, EXT);
    const uint32_t cp = lane_id() & (P.copies - 1);
    if (P.outputs & TP_OUT_CLOSE_HIST) atomicAdd(&cnt[close_bin(close) * P.copies + cp], 1ull);
    if (P.outputs & TP_OUT_LABEL_TABLE) atomicAdd(&cnt[B.table + idx * P.copies + cp], 1ull);
    if (P.outputs & TP_OUT_SPREAD_COUNT) spread += (P.spread_any && close <= P.spread_le) ? 1u : 0u;
    if (P.outputs & TP_OUT_OPEN_CLOSE) {
        const uint32_t t2 = h.t_pq + h.t_pr + h.t_qr - t1 - t3;  // exact in uint32 arithmetic mod 2^32
        atomicAdd(&cnt[B.oc + close_bin(t2 - t1) * 32 + close_bin(close)], 1ull);
    }
    if (EXT && (P.outputs & TP_OUT_MAX_EDGE)) {
        // Algorithm 3: vertex labels pairwise distinct; bin of the largest edge time
        if (h.l_p != h.l_q && h.l_q != h.l_r && h.l_p != h.l_r)
            atomicAdd(&cnt[B.maxe + min(t3 >> P.max_edge_shift, 1023u)], 1ull);
    }
    if (EXT && P.maxe_keys) {
        // Algorithm 3's exact counting set: the same triangles, every value kept
        if (h.l_p != h.l_q && h.l_q != h.l_r && h.l_p != h.l_r) maxe_count(P, t3);
    }
    if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE))
        atomicAdd(&cnt[B.deg + multiset_index(h.b_p, h.b_q, h.b_r)], 1ull);
    if (EXT && (P.outputs & TP_OUT_DIRECTED))
        atomicAdd(&cnt[B.dir + h.dtype], 1ull);
    return 1;
}

// Degree bin of rank x: the largest k with first[k] <= x (first[0] = 0 and
// first[] is non-decreasing, 32 entries).
__device__ __forceinline__ uint32_t degree_bin_of(const uint32_t *first, uint32_t x)
{
    uint32_t b = 0;
#pragma unroll
    for (uint32_t step = 16; step; step >>= 1)
        if (first[b + step] <= x) b += step;
    return b;
}

// Reduce one hit per lane (lanes with valid == false hold none) into the
// counters of every request slot of a multi-request pass.  Counts and spread
// counts are added once per wave; histogram and table bins per lane.
__device__ __forceinline__ void reduce_multi(const Hit &h, bool valid, unsigned long long *cnt, const SlotSpec *slots,
                                             uint32_t n_slots, uint32_t words, const uint16_t *lut, uint32_t lut_shift,
                                             bool labels)
{
    const uint32_t t1 = min(min(h.t_pq, h.t_pr), h.t_qr);
    const uint32_t t3 = max(max(h.t_pq, h.t_pr), h.t_qr);
    const uint32_t close = t3 - t1;
    const uint32_t bin = close_bin(close);
    const uint32_t idx = (labels && valid) ? lut[(((h.l_p << lut_shift) | h.l_q) << lut_shift) | h.l_r] : 0u;
    const bool lane0 = lane_id() == 0;
    for (uint32_t s = 0; s < n_slots; ++s) {
        const SlotSpec &S = slots[s];
        if (S.off) continue;
        unsigned long long *c = cnt + (size_t)s * words;
        bool pass = valid;
        if (S.filters & TP_FILT_WINDOW)
            pass = pass && !S.window_empty && h.t_pq >= S.t_lo && h.t_pq <= S.t_hi && h.t_pr >= S.t_lo &&
                   h.t_pr <= S.t_hi && h.t_qr >= S.t_lo && h.t_qr <= S.t_hi;
        if (S.filters & TP_FILT_LABEL_MASK) pass = pass && ((S.label_mask[idx >> 6] >> (idx & 63)) & 1ull);
        const uint64_t m = __ballot(pass);
        if (!m) continue;
        if (lane0) atomicAdd(&c[TP_BW_TRIANGLES], (unsigned long long)__popcll(m));
        if (S.outputs & TP_OUT_SPREAD_COUNT) {
            const uint64_t m2 = __ballot(pass && S.spread_any && close <= S.spread_le);
            if (lane0 && m2) atomicAdd(&c[TP_BW_SPREAD], (unsigned long long)__popcll(m2));
        }
        if ((S.outputs & TP_OUT_CLOSE_HIST) && pass) atomicAdd(&c[TP_BW_HIST + bin], 1ull);
        if ((S.outputs & TP_OUT_LABEL_TABLE) && pass) atomicAdd(&c[TP_BW_TABLE + idx], 1ull);
    }
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

// Load through the constant address space: with a wave-uniform address this
// is a scalar load into SGPRs (the arrays are not written by the survey).
template <class T>
__device__ __forceinline__ T sload(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "scalar loads move whole dwords");
    typedef const __attribute__((address_space(4))) uint32_t *cptr;
    const cptr c = reinterpret_cast<cptr>(reinterpret_cast<uintptr_t>(p));
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) w[i] = c[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// In-edge records as loaded: key (q << kbits) | k (or a piece's record) and
// payload.  A block holds one in-edge per lane.
struct KeyBlock {
    uint64_t key;
    uint32_t pay;
};

// Loaded values are kept as loaded (no arithmetic on them until they are
// read), so that no instruction waits for a load right after issuing it.
struct RecBlock {
    uint64_t key;   // (q << kbits) | k
    uint32_t pay;   // rest of p's row | label(p) << 24
    uint32_t t_pq;  // time(p, q)
    uint32_t p;     // rank of p (enumeration)
};

// LOG_SLOTS > 0: LDS hash of Adj+(q) with 2^LOG_SLOTS slots at most.
// LOG_SLOTS == 0: binary search of Adj+(q) in HBM.
// WAVE == false: the BLOCK threads of a workgroup share one target's table
// and the records of a tile are dealt to its waves round-robin.
// WAVE == true: every wave is its own group, with its own table, tiles and
// counters, and never waits for the other waves (for small targets, whose
// tiles are too short to keep a whole workgroup busy between barriers).
// A wave walks its records in rows of up to 64 consecutive candidates of one
// pivot's row (lane i takes candidate i), so every address is a wave-uniform
// base plus the lane.  Hits go to a per-wave ring in LDS and are reduced 64
// at a time.
// FORM: kFormSurvey for the reductions above; kFormExt adds the extended
// reductions (max-edge bins, degree table), compiled into their own kernels
// so that the others keep their register budget; kFormPart counts the
// triangles at every edge (local participation) instead of reducing them.
// PIECES: the huge class, whose tiles each hold one piece of Adj+(q) and
// walk records cut to it (the other classes compile without this).
// The per-wave form of the plain survey is held to 64 registers, 8 waves
// per SIMD: its short tiles wait on chains of dependent loads, and more
// waves hide them (20,000-graph batch survey 539.6 -> 515.3 ms).
template <int LOG_SLOTS, int BLOCK, bool WAVE, bool META, bool ENUM, bool MULTI, int FORM, bool PIECES, bool WIDE>
__global__ __launch_bounds__(BLOCK, (WAVE && FORM == kFormSurvey && !ENUM) ? 8 : 1) void survey_kernel(SurveyParams P)
{
    constexpr int kSub = Depth<WAVE>::kSub;
    constexpr int kBatch = Depth<WAVE>::kBatch;
    constexpr uint32_t kChunkCand = Depth<WAVE>::kChunkCand;
    constexpr int kWaves = BLOCK / kWave;       // waves per workgroup
    constexpr int kW = WAVE ? 1 : kWaves;       // waves sharing one table
    constexpr int kGroup = WAVE ? kWave : BLOCK;  // threads sharing one table
    constexpr int kGroups = WAVE ? kWaves : 1;  // tables per workgroup
    const uint64_t kClaim = P.claim ? P.claim : 1u;  // tiles claimed at a time
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr uint32_t kSlots = LOG_SLOTS > 0 ? (2u << LOG_SLOTS) + kStash : 0u;
    // The per-wave form stages its table's keys (fewer than 2^LOG_SLOTS = 64,
    // so at most one per lane) with their times and labels in registers, so
    // the table costs one round trip to memory; the workgroup forms, whose
    // registers bound their occupancy, load the keys twice.
    constexpr bool kStage = WAVE && LOG_SLOTS > 0 && (1 << LOG_SLOTS) <= kGroup;
    // The per-wave tables of the plain survey (and of the multi-request
    // passes, whose hits carry the same items) walk eight records at a time,
    // one per group of kRecLanes lanes: records of tiny targets are short
    // (about 13 candidates in the 20,000-graph batch), so a 64-lane step per
    // record left most lanes idle and spent the step's scalar bookkeeping on
    // a handful of checks (the kernel was bound by scalar issue).
    constexpr bool kGroupWalk = WAVE && LOG_SLOTS > 0 && (FORM == kFormSurvey || FORM == kFormPart) && !ENUM && !PIECES;
    constexpr uint32_t kRecLanes = 8;  // lanes per record in that walk (16: batch survey 351 ms, 8: 349)
    static_assert(!MULTI || (META && !ENUM), "multi-request passes reduce metadata");
    constexpr bool EXT = FORM == kFormExt;
    constexpr bool PART = FORM == kFormPart;
    static_assert(!(EXT || PART) || (META && !ENUM && !MULTI), "extended forms are single-request metadata surveys");
    const uint32_t nc = counter_words<MULTI, FORM>(P);
    const bool kdir = EXT && P.dir_words;  // the directed census
    const bool kbins = EXT && (P.outputs & TP_OUT_DEGREE_TABLE);  // the degree table
    constexpr uint32_t kRingK = ring_size<WAVE, BLOCK, META, ENUM, MULTI, FORM, WIDE>();
    const LdsLayout L =
        lds_layout(kSlots * kGroups, META || ENUM, nc * kGroups, kWaves, P.lut_shift, PART, kdir, ENUM, kbins, kRingK);
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    const int grp = WAVE ? w : 0;     // this thread's group
    const int gtid = WAVE ? (int)lane_id() : tid;  // rank in the group
    const int wl = WAVE ? 0 : w;      // rank of this wave in the group
    uint32_t *hkey = reinterpret_cast<uint32_t *>(lds) + (size_t)grp * kSlots;
    uint32_t *hts = reinterpret_cast<uint32_t *>(lds + L.off_hts) + (size_t)grp * kSlots;
    uint8_t *hlab = lds + L.off_hlab + (size_t)grp * kSlots;
    uint8_t *hdir = lds + L.off_hdir + (size_t)grp * kSlots;  // EXT, directed census
    uint8_t *hbin = lds + L.off_hbin + (size_t)grp * kSlots;  // EXT, degree table: bin of each key
    uint32_t *hpos = reinterpret_cast<uint32_t *>(lds + L.off_hpos) + (size_t)grp * kSlots;  // PART; ENUM: ids
    uint32_t *hcnt = reinterpret_cast<uint32_t *>(lds + L.off_hcnt) + (size_t)grp * kSlots;  // PART
    unsigned long long *cnt_all = reinterpret_cast<unsigned long long *>(lds + L.off_cnt);
    unsigned long long *cnt = cnt_all + (size_t)grp * nc;
    uint16_t *lut = reinterpret_cast<uint16_t *>(lds + L.off_lut);
    __shared__ uint64_t mask_lds[13];
    __shared__ uint32_t dbin_lds[kGroups * 32];  // per group: the degree-bin bounds of its graph
    __shared__ uint8_t dtype_lds[EXT ? 64 : 1];
    __shared__ SlotSpec slot_lds[MULTI ? kMaxSlots : 1];
    __shared__ unsigned long long s_tile;
    __shared__ uint32_t s_stash_g[kGroups], s_fail_g[kGroups];
    uint32_t &s_stash = s_stash_g[grp];
    uint32_t &s_fail = s_fail_g[grp];
    // barrier of the threads that share a table
    auto gsync = [&]() {
        if (WAVE) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };

    const uint32_t lane = lane_id();
    uint4 *ring = reinterpret_cast<uint4 *>(lds + L.off_ring) + (size_t)w * kRingK;
    for (uint32_t i = tid; i < nc * kGroups; i += BLOCK) cnt_all[i] = 0;
    if (tid < 13) mask_lds[tid] = P.label_mask[tid];
    if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE))
        for (int i = tid; i < kGroups * 32; i += BLOCK) dbin_lds[i] = P.dbin_rank[i & 31];
    if (EXT && tid < 64) dtype_lds[tid] = P.dir_type[tid];
    if (MULTI) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(P.slots);
        uint32_t *dst = reinterpret_cast<uint32_t *>(slot_lds);
        for (uint32_t i = tid; i < P.n_slots * (sizeof(SlotSpec) / 4); i += BLOCK) dst[i] = src[i];
    }
    if (META) {
        const uint32_t ls = P.lut_shift, lm = (1u << ls) - 1;
        for (uint32_t i = tid; i < (1u << (3 * ls)); i += BLOCK)
            lut[i] = (uint16_t)multiset_index(i >> (2 * ls), (i >> ls) & lm, i & lm);
    }
    __syncthreads();

    unsigned long long my_tri = 0, my_spread = 0, probes = 0;
    uint32_t qh = 0, qt = 0;  // this wave's hit ring: entries [qh, qt)

    // merge this workgroup's counters into graph g's result block; every
    // thread of the workgroup calls it
    auto flush = [&](uint32_t g) {
        unsigned long long *blk = P.out + (size_t)g * P.g_stride;
        const unsigned long long t = wave_sum(my_tri), sp = wave_sum(my_spread);
        if (lane == 0 && !MULTI) {
            if (t) atomicAdd(&blk[P.o_tri], t);
            if (sp) atomicAdd(&blk[P.o_spread], sp);
            if (probes) atomicAdd(&blk[P.o_probes], probes);
        }
        my_tri = 0;
        my_spread = 0;
        probes = 0;
        gsync();
        for (uint32_t i = gtid; i < nc; i += kGroup) {
            const unsigned long long v = cnt[i];
            if (!v) continue;
            uint32_t word;
            if (MULTI) {
                // slot i / slot_words, at the same word of its block
                const uint32_t sl = i / P.slot_words;
                atomicAdd(&P.out[(size_t)sl * P.g_stride + (i - sl * P.slot_words)], v);
                cnt[i] = 0;
                continue;
            }
            const CounterBase B = counter_base(P, EXT);
            if (i < B.table) word = P.o_hist + i / P.copies;
            else if (i < B.oc) word = P.o_table + (i - B.table) / P.copies;
            else if (!EXT || i < B.maxe) word = P.o_oc + (i - B.oc);
            else if (i < B.deg) word = P.o_maxe + (i - B.maxe);
            else if (i < B.dir) word = P.o_deg + (i - B.deg);
            else word = P.o_dir + (i - B.dir);
            atomicAdd(&blk[word], v);
            cnt[i] = 0;
        }
        gsync();
    };
    uint32_t cur_g = 0;  // graph whose counters the workgroup holds
    uint64_t cur_tile = 0;  // global index of the tile being walked (enumeration)

    // the target whose out-list is in the LDS table, and its geometry
    uint32_t cur_q = 0xffffffffu, cur_piece = 0;
    uint32_t bin_q = 0;  // degree bin of cur_q (extended form, degree table)
    uint32_t id_q = 0;  // original id of cur_q (enumeration)
    uint64_t kq = 0;
    uint32_t dq = 0, l_q = 0, log_s = 0;
    uint32_t pk0 = 0, pn = 0;  // the table holds Adj+(q) slots [kq + pk0, kq + pk0 + pn)
    uint32_t n_stash = 0;  // keys in the stash
    bool gmode = LOG_SLOTS == 0;  // search Adj+(q) in HBM (huge targets, or a failed table)
    uint32_t *dbin_g = dbin_lds + grp * 32;
    // degree bin cursor of the pivots this wave walks: bin pb spans CSR slots [pb_lo, pb_hi)
    // (bounds of the graph whose tiles the group walks: 32 per graph of a batch)
    uint32_t pb = 0;
    uint64_t pb_lo = 0, pb_hi = ~0ull;
    if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE)) pb_hi = sload(P.dbin_slot + 1);

    // reduce the hits queued in this wave's ring, one per lane; `gm` says
    // where Adj+^m(q) is (true: HBM) at compile time, so that the table path
    // holds no global load
    auto drain = [&](uint32_t count, auto gm) {
        constexpr bool G = decltype(gm)::value;
        uint32_t tri = 0, spread = 0;
        Hit h{0, 0, 0, 0, 0, 0, 0, 0, 0};
        uint32_t e_p = 0, e_r = 0;  // original ids of p and r (enumeration)
        const bool valid = lane < count;
        if (valid) {
            const uint4 e = ring[(qh + lane) & (kRingK - 1)];
            const uint32_t where = e.x & 0x3fffffu;
            h.t_pq = e.z;
            h.l_p = e.x >> 22;
            h.l_q = l_q;
            h.t_pr = e.y;
            if constexpr (!G) {
                h.t_qr = hts[where];
                h.l_r = hlab[where];
            } else {
                h.t_qr = P.ets[kq + where];
                h.l_r = P.tlab[kq + where];
            }
            if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE)) {
                // the ring's last word holds the pivot's degree bin; the
                // table keeps that of every key
                h.b_p = e.w & 0xffu;
                h.b_q = bin_q;
                h.b_r = !G ? hbin[where] : degree_bin_of(dbin_g, P.col[kq + where]);
            }
            if (kdir) {
                // ... and the directions of (p, q) and (p, r) above it
                const uint32_t dqr = !G ? hdir[where] : P.edir[kq + where];
                h.dtype = dtype_lds[(((e.w >> 8) & 3u) << 4) | (((e.w >> 10) & 3u) << 2) | (dqr & 3u)];
            }
            if (ENUM) {
                // original ids: of r from the table (or through the CSR in
                // HBM), of p from the ring
                e_r = !G ? hpos[where] : P.perm[P.col[kq + where]];
                e_p = e.w;
            } else if (!MULTI) {
                tri = reduce_hit<EXT, WAVE>(P, h, cnt, mask_lds, lut, spread);
            }
        }
        if (ENUM) {
            // the wave's records that pass the prefilters take consecutive
            // places, claimed with one atomic
            const bool pass = valid && (!P.filters || passes_filters<WAVE>(P, h, mask_lds, lut));
            const uint64_t vm = __ballot(pass);
            if (vm) {
                const unsigned k = (unsigned)__popcll(vm);
                unsigned long long base = 0;
                if (lane == 0) {
                    if (P.enum_tile_count) atomicAdd(&P.enum_tile_count[cur_tile], k);
                    else if (P.enum_tile_base)
                        base = P.enum_tile_base[cur_tile] - P.enum_chunk_base + atomicAdd(&P.enum_tile_cursor[cur_tile], k);
                    else base = atomicAdd(P.enum_count, (unsigned long long)k);
                }
                // (the builtin returns a signed int: each half is widened as unsigned)
                base = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)base);
                const unsigned long long at =
                    base + __builtin_amdgcn_mbcnt_hi((uint32_t)(vm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)vm, 0u));
                if (pass && !P.enum_tile_count && at < P.enum_cap) {
                    uint32_t *o = P.enum_out + at * 9;
                    o[0] = e_p;
                    o[1] = id_q;
                    o[2] = e_r;
                    o[3] = h.t_pq;
                    o[4] = h.t_pr;
                    o[5] = h.t_qr;
                    o[6] = h.l_p;
                    o[7] = h.l_q;
                    o[8] = h.l_r;
                }
            }
            tri = pass ? 1u : 0u;
        }
        if (MULTI) reduce_multi(h, valid, cnt, slot_lds, P.n_slots, P.slot_words, lut, P.lut_shift, P.slot_labels);
        my_tri += tri;
        my_spread += spread;
        qh = __builtin_amdgcn_readfirstlane(qh + count);
    };
    // reduce 128 queued hits, two per lane (the doubled ring of the plain
    // survey): both hits' reads are issued before either is reduced.  The
    // wave runs it at raised priority, so that its chains of LDS reads and
    // adds issue ahead of the other waves' probing (large class 309.3 ->
    // 302.1 ms; priority 3 no better, and the same for the one-hit drains of
    // the other kernels slowed the batch survey)
    auto drain2 = [&](auto gm) {
        constexpr bool G = decltype(gm)::value;
        __builtin_amdgcn_s_setprio(2);
        const uint4 e0 = ring[(qh + lane) & (kRingK - 1)];
        const uint4 e1 = ring[(qh + kWave + lane) & (kRingK - 1)];
        const uint32_t w0 = e0.x & 0x3fffffu, w1 = e1.x & 0x3fffffu;
        Hit h0{e0.z, e0.y, 0, e0.x >> 22, l_q, 0, 0, 0, 0, 0};
        Hit h1{e1.z, e1.y, 0, e1.x >> 22, l_q, 0, 0, 0, 0, 0};
        if constexpr (!G) {
            h0.t_qr = hts[w0];
            h1.t_qr = hts[w1];
            h0.l_r = hlab[w0];
            h1.l_r = hlab[w1];
        } else {
            h0.t_qr = P.ets[kq + w0];
            h1.t_qr = P.ets[kq + w1];
            h0.l_r = P.tlab[kq + w0];
            h1.l_r = P.tlab[kq + w1];
        }
        uint32_t spread = 0;
        uint32_t tri = reduce_hit<EXT, WAVE>(P, h0, cnt, mask_lds, lut, spread);
        tri += reduce_hit<EXT, WAVE>(P, h1, cnt, mask_lds, lut, spread);
        my_tri += tri;
        my_spread += spread;
        qh = __builtin_amdgcn_readfirstlane(qh + 2 * kWave);
        __builtin_amdgcn_s_setprio(0);
    };
    auto drain_queued = [&]() {
        if constexpr (kRingK > kRing) {
            // the doubled ring may hold more than a wave's 64
            while (qt - qh > (uint32_t)kWave) {
                if (gmode) drain(kWave, std::true_type{});
                else drain(kWave, std::false_type{});
            }
        }
        if (qt == qh) return;
        if (gmode) drain(qt - qh, std::true_type{});
        else drain(qt - qh, std::false_type{});
    };
    // participation: add the table's per-slot counts of edges (q, r) into
    // their CSR slots; every thread of the group calls it once the group is
    // done with the table
    auto flush_part = [&]() {
        if (!PART || LOG_SLOTS == 0 || cur_q == 0xffffffffu || gmode) return;
        const uint32_t top = (2u << log_s) + n_stash;
        for (uint32_t h = gtid; h < top; h += kGroup) {
            if (hkey[h] == kEmpty) continue;
            const uint32_t c = hcnt[h];
            if (c) atomicAdd(&P.part_edge[kq + hpos[h]], (unsigned long long)c);
        }
    };

    // this workgroup's segment of the launch's tiles first, then the others
    const uint32_t nseg = 1u << P.claim_seg_log;
    uint32_t seg = blockIdx.x & (nseg - 1);
    uint32_t segs_left = nseg;
    uint64_t seg_lo = (P.n_tiles * seg) >> P.claim_seg_log;
    uint64_t seg_hi = (P.n_tiles * (seg + 1)) >> P.claim_seg_log;
    for (;;) {
        // claim a chunk of kClaim consecutive tiles; consecutive tiles mostly
        // share their target, whose table is then built once
        uint64_t t_begin;
        if (WAVE) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(P.tile_counter + seg, 1ull);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)c);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(c >> 32));
            t_begin = seg_lo + (((uint64_t)hi << 32) | lo) * kClaim;
        } else {
            if (tid == 0) s_tile = atomicAdd(P.tile_counter + seg, 1ull);
            __syncthreads();
            t_begin = seg_lo + s_tile * kClaim;
            __syncthreads();  // everyone has read s_tile before it is claimed again
        }
        if (t_begin >= seg_hi) {
            // the segment is used up (its counter only grows): the next one
            if (--segs_left == 0) break;
            seg = (seg + 1) & (nseg - 1);
            seg_lo = (P.n_tiles * seg) >> P.claim_seg_log;
            seg_hi = (P.n_tiles * (seg + 1)) >> P.claim_seg_log;
            continue;
        }
        const uint64_t t_end = min(t_begin + kClaim, seg_hi);
        for (uint64_t ti = t_begin; ti < t_end; ++ti) {
            const TileDesc d = sload(P.tiles + (P.n_tiles - 1 - ti));
            if (ENUM) cur_tile = P.tile_gbase + (P.n_tiles - 1 - ti);
            // this wave's records: tile records wl, wl + kW, wl + 2kW, ...;
            // lane l of block b holds record 64b + l.  The first two blocks
            // are requested before the table is rebuilt, so that their
            // latency hides behind it.  Lanes past the wave's last record
            // load the tile's first record; they are never read.
            const uint32_t ncnt = d.cnt;
            const uint32_t nw = ncnt > (uint32_t)wl ? (ncnt - (uint32_t)wl + kW - 1) / kW : 0u;
            auto load_keys = [&](uint32_t blk) -> KeyBlock {
                const uint32_t i = min(blk * kWave + lane, nw - 1);
                const uint64_t e = d.e0 + ((uint64_t)(uint32_t)wl + (uint64_t)i * kW) * d.stride;
                return KeyBlock{P.inkey[e], P.inpay[e]};
            };
            KeyBlock kb0{0, 0}, kb1{0, 0};
            if (nw) {
                kb0 = load_keys(0);
                kb1 = load_keys(1);
            }
            if (d.q != cur_q || (PIECES && d.piece != cur_piece)) {
                // a new target (or piece): reduce the hits still queued
                // against the old table, then rebuild it once every wave is
                // done with it
                if (META || ENUM) drain_queued();
                if (P.rank_gid) {
                    const uint32_t g = sload(P.rank_gid + d.q);
                    if (g != cur_g) {
                        flush(cur_g);
                        cur_g = g;
                        if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE)) {
                            // the new graph's degree-bin bounds (published by
                            // the barrier below) and a fresh pivot cursor
                            for (uint32_t i = gtid; i < 32; i += kGroup) dbin_g[i] = P.dbin_rank[(size_t)g * 32 + i];
                            pb = 0;
                            pb_lo = 0;
                            pb_hi = sload(P.dbin_slot + (size_t)g * 32 + 1);
                        }
                    }
                }
                gsync();
                if (PART) {
                    flush_part();
                    gsync();
                }
                cur_q = d.q;
                cur_piece = d.piece;
                kq = sload(P.rowptr + cur_q);
                dq = (uint32_t)(sload(P.rowptr + cur_q + 1) - kq);
                l_q = META ? __builtin_amdgcn_readfirstlane(P.rlab[cur_q]) : 0u;
                if (ENUM) id_q = sload(P.perm + cur_q);
                if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE))
                    bin_q = __builtin_amdgcn_readfirstlane(degree_bin_of(dbin_g, cur_q));
                pk0 = PIECES ? min(cur_piece, piece_count(dq)) * piece_size(dq) : 0u;
                pn = PIECES ? (pk0 < dq ? min(dq - pk0, piece_size(dq)) : 0u) : dq;
                log_s = 5;
                while ((1u << log_s) < pn + pn / 4) ++log_s;
                // a target too large for this kernel's tables (the planner's
                // classes never send one) is searched in HBM
                if (LOG_SLOTS > 0) gmode = log_s > (uint32_t)LOG_SLOTS;
                if (LOG_SLOTS > 0 && !gmode) {
                    // two tables of 2^log_s >= 1.25 dq slots each, then the stash.
                    // Staged keys, times and labels are requested before the
                    // clearing, which their latency overlaps.
                    const uint32_t S = 1u << log_s;
                    uint32_t kcol = kEmpty, kts = 0, klab = 0;  // this lane's key (gtid < pn), staged
                    if (kStage && gtid < pn) {
                        kcol = P.col[kq + pk0 + gtid];
                        if (META || ENUM) {
                            kts = P.ets[kq + pk0 + gtid];
                            klab = P.tlab[kq + pk0 + gtid];
                        }
                    }
                    for (uint32_t i = gtid; i < 2 * S + kStash; i += kGroup) hkey[i] = kEmpty;
                    if (gtid == 0) {
                        s_stash = 0;
                        s_fail = 0;
                    }
                    gsync();
                    // cuckoo insertion: a key evicted from one table moves to
                    // its slot in the other; keys still homeless after
                    // kMaxKicks moves go to the stash
                    for (uint32_t i = gtid; i < pn; i += kGroup) {
                        uint32_t cur = kStage ? kcol : P.col[kq + pk0 + i];
                        uint32_t t = 0;
                        for (uint32_t it = 0; it < P.max_kicks; ++it) {
                            const uint32_t h = t == 0 ? hash0(cur, log_s) : S + hash1(cur, log_s);
                            cur = atomicExch(&hkey[h], cur);
                            if (cur == kEmpty) break;
                            t ^= 1u;
                        }
                        if (cur != kEmpty) {
                            const uint32_t at = atomicAdd(&s_stash, 1u);
                            if (at < kStash) hkey[2 * S + at] = cur;
                            else s_fail = 1;
                        }
                    }
                    gsync();
                    n_stash = __builtin_amdgcn_readfirstlane(min(s_stash, kStash));
                    gmode = __builtin_amdgcn_readfirstlane(s_fail) != 0;
                    // the metadata of every key goes beside its final slot
                    if ((META || ENUM) && !gmode) {
                        for (uint32_t i = gtid; i < pn; i += kGroup) {
                            const uint32_t r = kStage ? kcol : P.col[kq + pk0 + i];
                            uint32_t h = hash0(r, log_s);
                            if (hkey[h] != r) {
                                h = S + hash1(r, log_s);
                                if (hkey[h] != r) {
                                    h = 2 * S;
                                    while (hkey[h] != r) ++h;
                                }
                            }
                            hts[h] = kStage ? kts : P.ets[kq + pk0 + i];
                            hlab[h] = kStage ? (uint8_t)klab : P.tlab[kq + pk0 + i];
                            if (PART) {
                                hpos[h] = pk0 + i;
                                hcnt[h] = 0;
                            }
                            if (kdir) hdir[h] = P.edir[kq + pk0 + i];
                            if (kbins) hbin[h] = (uint8_t)degree_bin_of(dbin_g, r);
                            if (ENUM) hpos[h] = P.perm[r];
                        }
                    }
                }
                gsync();
            }

            // ---- this wave's records: tile records w, w + kW, w + 2kW, ...,
            // walked with the search mode fixed at compile time (see drain).
            // The wave loads them 64 at a time into VGPRs (lane i holds its
            // i-th record) and reads the current one with readlane, so the
            // walk itself issues no memory access.
            auto walk = [&](auto gm) {
                constexpr bool G = decltype(gm)::value;
                if (nw == 0) return;
                const uint64_t kmask = (1ull << P.kbits) - 1;
                // A block is loaded in two stages a block apart, so that no
                // load waits on a load issued just before it (loads retire in
                // order: such a wait would drain the candidate loads in
                // flight): the records of block b + 2, then the gather of
                // time(p, q) for block b + 1 from keys that arrived long ago.
                auto gather = [&](const KeyBlock &kb) -> RecBlock {
                    RecBlock r;
                    r.key = kb.key;
                    r.pay = kb.pay;
                    r.t_pq = (META || ENUM) ? P.ets[kb.key & kmask] : 0u;
                    r.p = ENUM ? P.enum_srow[kb.key & kmask] : 0u;
                    if (PIECES && !PART && !kdir) {
                        // a record cut to a piece: once its slot's gathers
                        // are issued, the slot moves past the skipped
                        // candidates, still in p's row (participation and the
                        // directed census, which need the slot of p -> q
                        // later, skip them record by record)
                        r.key = (kb.key & kmask) + ((kb.key >> P.kbits) - cur_q);
                    }
                    return r;
                };
                RecBlock blk_cur = gather(kb0);
                RecBlock blk_nxt = gather(kb1);
                KeyBlock key_nxt = load_keys(2);
                if constexpr (kGroupWalk && !G) {
                    // ---- 64 / kRecLanes records at a time: lanes
                    // [kRecLanes u, kRecLanes (u + 1)) walk one record,
                    // kRecLanes candidates a step, and take the next record
                    // once their own is done
                    const uint32_t sub = lane & (kRecLanes - 1);
                    const uint32_t lead = lane & ~(kRecLanes - 1);  // the group's first lane
                    const uint64_t lower = (1ull << lead) - 1ull;  // lanes of the groups below
                    uint32_t cb = 0;    // block held in blk_cur: records 64 cb .. 64 cb + 63
                    uint32_t next = 0;  // records handed out
                    uint64_t qs = 0;    // this group's next candidate slot
                    uint32_t qleft = 0, qtpq = 0, qlp = 0;  // its candidates left, time(p, q), label(p)
                    uint64_t qpq = 0;   // slot of p -> q (participation)
                    uint32_t wave_work = 0, wave_hits = 0;
                    // groups without a record take the next ones, in order
                    auto refill = [&]() {
                        const uint64_t need = __ballot(sub == 0 && qleft == 0);
                        if (need == 0 || next >= nw) return;
                        const uint32_t k = (uint32_t)__popcll(need);
                        const uint32_t j = next + (uint32_t)__popcll(need & lower);
                        const uint32_t src = j & (kWave - 1);
                        uint32_t klo = __shfl((uint32_t)blk_cur.key, (int)src);
                        uint32_t khi = __shfl((uint32_t)(blk_cur.key >> 32), (int)src);
                        uint32_t pay = __shfl(blk_cur.pay, (int)src);
                        uint32_t tpq = __shfl(blk_cur.t_pq, (int)src);
                        if (((next + k - 1) >> 6) != cb) {
                            // some of them are in the next block
                            const uint32_t nlo = __shfl((uint32_t)blk_nxt.key, (int)src);
                            const uint32_t nhi = __shfl((uint32_t)(blk_nxt.key >> 32), (int)src);
                            const uint32_t npay = __shfl(blk_nxt.pay, (int)src);
                            const uint32_t ntpq = __shfl(blk_nxt.t_pq, (int)src);
                            if ((j >> 6) != cb) {
                                klo = nlo;
                                khi = nhi;
                                pay = npay;
                                tpq = ntpq;
                            }
                        }
                        if (((need >> lead) & 1ull) && j < nw) {
                            qs = ((((uint64_t)khi << 32) | klo) & kmask) + 1;
                            qpq = qs - 1;
                            qleft = pay & 0xffffffu;
                            qtpq = tpq;
                            qlp = pay >> 24;
                        }
                        next = min(next + k, nw);
                        if (next >= 64u * (cb + 1u) && next < nw) {
                            blk_cur = blk_nxt;
                            blk_nxt = gather(key_nxt);
                            key_nxt = load_keys(cb + 3u);
                            ++cb;
                        }
                    };
                    struct Step {
                        uint32_t cand, tpr, tpq, lp;
                        uint64_t live;
                        uint64_t pr, pq;  // participation: slots of (p, r) and of p -> q
                    };
                    // request the next kRecLanes candidates of every group's record
                    auto issue = [&](Step &st) -> bool {
                        const uint32_t n = min(qleft, kRecLanes);
                        const bool lv = sub < n;
                        st.live = __ballot(lv);
                        if (st.live == 0) return false;
                        st.cand = 0;
                        st.tpr = 0;
                        if (lv) {
                            st.cand = P.col[qs + sub];
                            if (META) st.tpr = P.ets[qs + sub];
                        }
                        st.tpq = qtpq;
                        st.lp = qlp;
                        if constexpr (PART) {
                            st.pr = qs + sub;
                            st.pq = qpq;
                        }
                        wave_work += (uint32_t)__popcll(st.live);
                        qs += n;
                        qleft -= n;
                        return true;
                    };
                    auto probe = [&](const Step &st) {
                        const uint32_t r = st.cand;
                        const uint32_t h0 = hash0(r, log_s), h1 = (1u << log_s) + hash1(r, log_s);
                        const uint32_t k0 = hkey[h0], k1 = hkey[h1];
                        bool hit = k0 == r || k1 == r;
                        uint32_t slot = k0 == r ? h0 : h1;
                        if (n_stash) {
                            const uint32_t st0 = 2u << log_s;
                            for (uint32_t x = 0; x < n_stash; ++x) {
                                if (hkey[st0 + x] == r) {
                                    hit = true;
                                    slot = st0 + x;
                                }
                            }
                        }
                        const uint64_t m = __ballot(hit) & st.live;
                        if (!META) {
                            wave_hits += (uint32_t)__popcll(m);
                            return;
                        }
                        if constexpr (PART) {
                            // one count for each edge of every triangle that
                            // passes the prefilters: (p, r) by its slot, (q, r)
                            // per table slot, (p, q) once per record group
                            bool pass = (m >> lane) & 1ull;
                            if (pass && P.filters) {
                                Hit h{st.tpq, st.tpr, hts[slot], st.lp, l_q, hlab[slot], 0, 0, 0, 0};
                                pass = passes_filters<WAVE>(P, h, mask_lds, lut);
                            }
                            const uint64_t pm = __ballot(pass);
                            if (pass) {
                                atomicAdd(&P.part_edge[st.pr], 1ull);
                                atomicAdd(&hcnt[slot], 1u);
                            }
                            const uint64_t gm_mask = (kRecLanes == 64 ? ~0ull : ((1ull << kRecLanes) - 1)) << lead;
                            const uint32_t in_group = (uint32_t)__popcll(pm & gm_mask);
                            if (sub == 0 && in_group) atomicAdd(&P.part_edge[st.pq], (unsigned long long)in_group);
                            wave_hits += (uint32_t)__popcll(pm);
                            return;
                        }
                        if (m) {
                            if ((m >> lane) & 1ull) {
                                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                                ring[(qt + below) & (kRingK - 1)] = make_uint4(slot | (st.lp << 22), st.tpr, st.tpq, 0u);
                            }
                            qt = __builtin_amdgcn_readfirstlane(qt + (uint32_t)__popcll(m));
                            if (qt - qh >= (uint32_t)kWave) drain(kWave, gm);
                        }
                    };
                    // two steps in flight: the next step's loads are issued
                    // before the current one is probed
                    Step sa, sb;
                    refill();
                    if (issue(sa)) {
                        for (;;) {
                            refill();
                            const bool more_b = issue(sb);
                            probe(sa);
                            if (!more_b) break;
                            refill();
                            const bool more_a = issue(sa);
                            probe(sb);
                            if (!more_a) break;
                        }
                    }
                    if (lane == 0) {
                        probes += wave_work;
                        my_tri += wave_hits;
                    }
                    return;
                }
                struct WaveRec {
                    uint64_t k, start;  // slot of p -> q, first candidate
                    uint32_t len, t_pq, l_p, p;
                };
                auto read_rec = [&](uint32_t i) -> WaveRec {
                    const uint32_t l = i & (kWave - 1);
                    WaveRec r;
                    const uint64_t key = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)blk_cur.key, l) |
                                         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(blk_cur.key >> 32), l)
                                          << 32);
                    const uint32_t pay = __builtin_amdgcn_readlane(blk_cur.pay, l);
                    r.start = (key & kmask) + 1;
                    r.k = r.start - 1;
                    if (PIECES && (PART || kdir)) r.start += (key >> P.kbits) - cur_q;
                    r.len = pay & 0xffffffu;
                    r.t_pq = (META || ENUM) ? __builtin_amdgcn_readlane(blk_cur.t_pq, l) : 0;
                    r.l_p = (META || ENUM) ? pay >> 24 : 0;
                    r.p = 0;
                    if (EXT && (P.outputs & TP_OUT_DEGREE_TABLE)) {
                        // degree bin of the pivot, from a slot of p's row (that
                        // of p -> q, or past it for a record cut to a piece):
                        // a wave meets its records in increasing slot order
                        // within a tile, so the bin cursor mostly moves forward
                        const uint64_t s0 = r.k;
                        const uint64_t *dslot = P.dbin_slot + (size_t)cur_g * 32;
                        if (s0 < pb_lo) {
                            pb = 0;
                            pb_lo = 0;
                            pb_hi = sload(dslot + 1);
                        }
                        while (s0 >= pb_hi) {
                            ++pb;
                            pb_lo = pb_hi;
                            pb_hi = pb < 31 ? sload(dslot + pb + 1) : ~0ull;
                        }
                        r.p = pb;
                    }
                    if (kdir) {
                        // direction of p -> q: the byte at slot k, read
                        // through the dword that holds it
                        const uint64_t s0 = r.k;
                        const uint32_t wd = sload(reinterpret_cast<const uint32_t *>(P.edir + (s0 & ~3ull)));
                        r.p |= ((wd >> ((uint32_t)(s0 & 3ull) * 8u)) & 3u) << 8;
                    }
                    if (ENUM) {
                        // the pivot's original id: its rank came with the
                        // record's other gathers
                        r.p = sload(P.perm + (uint32_t)__builtin_amdgcn_readlane(blk_cur.p, l));
                    }
                    return r;
                };
                uint32_t i = 0;   // current record (wave-local index)
                WaveRec rec = read_rec(0);
                uint32_t off = 0; // next slot of the current record
                uint32_t wave_work = 0, wave_hits = 0;

                // next chunk of up to kChunkCand candidates of the current
                // record: its size and the record's metadata; returns the
                // chunk's first slot
                struct Chunk {
                    uint32_t n, t_pq, l_p, p;
                    uint64_t base, spq;  // slot of the first candidate, and of p -> q (participation)
                };
                auto next_chunk = [&](Chunk &ch) -> uint64_t {
                    uint64_t base = 0;
                    if (i < nw) {
                        base = rec.start + off;
                        ch.n = min(rec.len - off, kChunkCand);
                        ch.t_pq = rec.t_pq;
                        ch.l_p = rec.l_p;
                        ch.p = rec.p;
                        ch.base = base;
                        ch.spq = rec.k;
                        wave_work += ch.n;
                        off += kChunkCand;
                        if (off >= rec.len) {
                            off = 0;
                            ++i;
                            if (i < nw) {
                                if ((i & (kWave - 1)) == 0) {
                                    blk_cur = blk_nxt;
                                    blk_nxt = gather(key_nxt);
                                    key_nxt = load_keys(i / kWave + 2);
                                }
                                rec = read_rec(i);
                            }
                        }
                    } else {
                        ch.n = 0;
                        ch.t_pq = 0;
                        ch.l_p = 0;
                        ch.p = 0;
                        ch.base = 0;
                        ch.spq = 0;
                    }
                    return base;
                };
                // issue the loads of kBatch chunks: lane l of sub-row s reads
                // candidate 64 s + l; the buffer resource spans exactly the
                // chunk, so lanes past its end read 0 without touching memory
                auto prepare = [&](Chunk(&chs)[kBatch], uint32_t(&cand)[kBatch][kSub], uint32_t(&tpr)[kBatch][kSub],
                                   uint32_t(&dpr)[kBatch][kSub]) {
    #pragma unroll
                    for (int c = 0; c < kBatch; ++c) {
                        const uint64_t base = next_chunk(chs[c]);
                        const uint32_t bytes = chs[c].n * 4u;
                        const auto rc = __builtin_amdgcn_make_buffer_rsrc((void *)(P.col + base), (short)0, bytes, kRsrcWord3);
    #pragma unroll
                        for (int sr = 0; sr < kSub; ++sr)
                            cand[c][sr] = __builtin_amdgcn_raw_buffer_load_b32(rc, lane * 4u + sr * 256u, 0, 0);
                        if (META || ENUM) {
                            const auto rt =
                                __builtin_amdgcn_make_buffer_rsrc((void *)(P.ets + base), (short)0, bytes, kRsrcWord3);
    #pragma unroll
                            for (int sr = 0; sr < kSub; ++sr)
                                tpr[c][sr] = __builtin_amdgcn_raw_buffer_load_b32(rt, lane * 4u + sr * 256u, 0, 0);
                        }
                        if constexpr (EXT) {
                            if (kdir) {
                                // directions of (p, r), one byte per candidate
                                const auto rd = __builtin_amdgcn_make_buffer_rsrc((void *)(P.edir + base), (short)0,
                                                                                  chs[c].n, kRsrcWord3);
    #pragma unroll
                                for (int sr = 0; sr < kSub; ++sr)
                                    dpr[c][sr] = __builtin_amdgcn_raw_buffer_load_b8(rd, lane + sr * 64u, 0, 0);
                            }
                        }
                    }
                };
                auto process = [&](const Chunk(&chs)[kBatch], const uint32_t(&cand)[kBatch][kSub],
                                   const uint32_t(&tpr)[kBatch][kSub], const uint32_t(&dpr)[kBatch][kSub]) {
    #pragma unroll
                    for (int c = 0; c < kBatch; ++c) {
    #pragma unroll
                        for (int sr = 0; sr < kSub; ++sr) {
                            if constexpr (kRingK > kRing) {
                                // the doubled ring takes two sub-rows of hits (at most
                                // 128) above 127 queued: drained before every other
                                // sub-row only, so that the unrolled walk holds half
                                // the copies of the reduction (large class 316.5 ->
                                // 311.5 ms)
                                if ((sr & 1) == 0 && qt - qh >= 2u * kWave) drain2(gm);
                            }
                            if (chs[c].n <= (uint32_t)(sr * kWave)) break;
                            const uint32_t nsub = min(chs[c].n - sr * kWave, (uint32_t)kWave);
                            // lanes >= nsub hold no candidate (they read 0): mask their hits
                            const uint64_t live = nsub >= (uint32_t)kWave ? ~0ull : ((1ull << nsub) - 1);
                            const uint32_t r = cand[c][sr];
                            bool hit;
                            uint32_t slot;
                            if constexpr (!G) {
                                // two independent reads, no loop
                                const uint32_t h0 = hash0(r, log_s), h1 = (1u << log_s) + hash1(r, log_s);
                                const uint32_t k0 = hkey[h0], k1 = hkey[h1];
                                hit = k0 == r || k1 == r;
                                slot = k0 == r ? h0 : h1;
                                if (n_stash) {
                                    const uint32_t st = 2u << log_s;
                                    for (uint32_t x = 0; x < n_stash; ++x) {
                                        if (hkey[st + x] == r) {
                                            hit = true;
                                            slot = st + x;
                                        }
                                    }
                                }
                            } else {
                                hit = false;
                                slot = 0;
                                if (lane < nsub) {
                                    const int64_t at = global_find(P.col, kq, dq, r);
                                    hit = at >= 0;
                                    slot = (uint32_t)(at - (int64_t)kq);
                                }
                            }
                            const uint64_t m = __ballot(hit) & live;
                            if constexpr (PART) {
                                // local participation: one count for each edge of
                                // every triangle that passes the prefilters
                                bool pass = (m >> lane) & 1ull;
                                if (pass && P.filters) {
                                    Hit h{chs[c].t_pq, tpr[c][sr], 0, chs[c].l_p, l_q, 0, 0, 0, 0};
                                    if constexpr (!G) {
                                        h.t_qr = hts[slot];
                                        h.l_r = hlab[slot];
                                    } else {
                                        h.t_qr = P.ets[kq + slot];
                                        h.l_r = P.tlab[kq + slot];
                                    }
                                    pass = passes_filters<WAVE>(P, h, mask_lds, lut);
                                }
                                const uint64_t pm = __ballot(pass);
                                if (pass) {
                                    atomicAdd(&P.part_edge[chs[c].base + (uint32_t)(sr * kWave) + lane], 1ull);  // (p, r)
                                    if constexpr (!G) atomicAdd(&hcnt[slot], 1u);  // (q, r), per table slot
                                    else atomicAdd(&P.part_edge[kq + slot], 1ull);
                                }
                                if (pm) {
                                    if (lane == 0) atomicAdd(&P.part_edge[chs[c].spq], (unsigned long long)__popcll(pm));
                                    wave_hits += (uint32_t)__popcll(pm);
                                }
                                continue;
                            }
                            if (!META && !ENUM) {
                                wave_hits += (uint32_t)__popcll(m);
                                continue;
                            }
                            if (m) {
                                if ((m >> lane) & 1ull) {
                                    // position among the wave's hits: hits in the lanes below
                                    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                                        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                                    ring[(qt + below) & (kRingK - 1)] =
                                        make_uint4(slot | (chs[c].l_p << 22), tpr[c][sr], chs[c].t_pq,
                                                   EXT && kdir ? chs[c].p | ((dpr[c][sr] & 3u) << 10) : chs[c].p);
                                }
                                // the ring cursors are wave-uniform: keep them in scalar registers
                                qt = __builtin_amdgcn_readfirstlane(qt + (uint32_t)__popcll(m));
                                if constexpr (kRingK == kRing) {
                                    if (qt - qh >= (uint32_t)kWave) drain(kWave, gm);
                                }
                            }
                        }
                    }
                };
                // two batches in flight: the next batch's loads are issued before
                // the current batch is probed
                Chunk rA[kBatch], rB[kBatch];
                uint32_t cA[kBatch][kSub], tA[kBatch][kSub], cB[kBatch][kSub], tB[kBatch][kSub];
                uint32_t dA[kBatch][kSub], dB[kBatch][kSub];  // extended form, directed census
                prepare(rA, cA, tA, dA);
                for (;;) {
                    prepare(rB, cB, tB, dB);
                    process(rA, cA, tA, dA);
                    if (rB[0].n == 0) break;
                    prepare(rA, cA, tA, dA);
                    process(rB, cB, tB, dB);
                    if (rA[0].n == 0) break;
                }
                if (lane == 0) {
                    probes += wave_work;
                    my_tri += wave_hits;
                }
            };
            if (gmode) walk(std::true_type{});
            else walk(std::false_type{});
            // a streamed or counted enumeration places records by tile: the
            // ring must not carry them into the next tile
            if (ENUM && (P.enum_tile_base || P.enum_tile_count)) drain_queued();
        }
    }

    if (META || ENUM) drain_queued();
    if (PART) {
        gsync();
        flush_part();
    }
    // ---- merge this workgroup's counters into the result
    flush(cur_g);
}

// dst = *src, by one thread (a snapshot of a counter between launches)
__global__ void k_copy_word(const unsigned long long *src, unsigned long long *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ void zero_u64(unsigned long long *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// The row (pivot rank) of every CSR slot, for enumeration: one wave per row.
__global__ void k_slot_rows(const uint64_t *rowptr, uint32_t n, uint32_t *srow)
{
    const size_t waves = (size_t)gridDim.x * blockDim.x / kWave;
    for (size_t v = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave; v < n; v += waves) {
        const uint64_t b = rowptr[v], e = rowptr[v + 1];
        for (uint64_t i = b + lane_id(); i < e; i += kWave) srow[i] = (uint32_t)v;
    }
}

void slot_rows(const tp_graph *g, DArray<uint32_t> &srow, hipStream_t s)
{
    srow.reset(std::max<uint64_t>(g->m, 1), s);
    if (!g->m) return;
    k_slot_rows<<<grid_for((size_t)g->n * kWave, 256), 256, 0, s>>>(g->rowptr.get(), g->n, srow.get());
    TP_CHECK_LAUNCH();
}

// Largest of n uint32 values into *out (zeroed by the caller).
__global__ void k_max_u32(const unsigned *x, size_t n, unsigned long long *out)
{
    unsigned long long mx = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        mx = max(mx, (unsigned long long)x[i]);
    mx = wave_max(mx);
    if (lane_id() == 0 && mx) atomicMax(out, mx);
}

// The next chunk of a streamed enumeration: the largest t1 > t0 with
// base[t1] - base[t0] <= cap (t0 itself when even one tile does not fit).
// Writes t1, base[t0], base[t1].
__global__ void k_enum_chunk(const uint64_t *base, uint64_t n_tiles, uint64_t t0, uint64_t cap, uint64_t *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint64_t b0 = base[t0];
    uint64_t lo = t0, hi = n_tiles;  // base[lo] - b0 <= cap; find the last such index
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (base[mid] - b0 <= cap) lo = mid;
        else hi = mid - 1;
    }
    out[0] = lo;
    out[1] = b0;
    out[2] = base[lo];
}

// Vertex participation from edge participation: each triangle at v holds
// two of v's edges, so twice v's count is the sum over its edges.  One wave
// per row adds each count to the edge's target and the row's sum to its
// source (a thread per row left hub rows to single threads).
__global__ void k_part_rows(const uint64_t *rowptr, const uint32_t *col, uint32_t n, const unsigned long long *edge,
                            unsigned long long *acc)
{
    const size_t waves = (size_t)gridDim.x * blockDim.x / kWave;
    for (size_t v = (blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave; v < n; v += waves) {
        const uint64_t b = rowptr[v], e = rowptr[v + 1];
        unsigned long long sum = 0;
        for (uint64_t i = b + lane_id(); i < e; i += kWave) {
            const unsigned long long c = edge[i];
            if (!c) continue;
            sum += c;
            atomicAdd(&acc[col[i]], c);
        }
        sum = wave_sum(sum);
        if (lane_id() == 0 && sum) atomicAdd(&acc[v], sum);
    }
}

__global__ void k_part_vertex(const unsigned long long *acc, const uint32_t *perm, uint32_t n, uint64_t *out)
{
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        out[perm[v]] = acc[v] / 2;
}

uint32_t table_size(uint32_t L) { return (L + 2) * (L + 1) * L / 6; }

// Dynamic LDS a workgroup may take: 160 KiB per compute unit, less room for
// the kernel's static arrays.
constexpr size_t kLdsLimit = 160 * 1024 - 4096;

template <int LOG_SLOTS, int BLOCK, bool WAVE, bool META, bool ENUM, bool MULTI, int FORM, bool WIDE = false>
size_t lds_need(const SurveyParams &P)
{
    constexpr uint32_t groups = WAVE ? BLOCK / kWave : 1;
    const uint32_t slots = LOG_SLOTS > 0 ? (2u << LOG_SLOTS) + kStash : 0u;
    const uint32_t nc = counter_words<MULTI, FORM>(P);
    return lds_layout(slots * groups, META || ENUM, nc * groups, BLOCK / kWave, P.lut_shift, FORM == kFormPart,
                      FORM == kFormExt && P.dir_words, ENUM,
                      FORM == kFormExt && (P.outputs & TP_OUT_DEGREE_TABLE),
                      ring_size<WAVE, BLOCK, META, ENUM, MULTI, FORM, WIDE>())
        .total;
}

template <int LOG_SLOTS, int BLOCK, bool WAVE, bool META, bool ENUM, bool MULTI, int FORM, bool PIECES, bool WIDE>
void launch_kernel(const SurveyParams &P, const LdsLayout &L, hipStream_t s, int device)
{
    constexpr uint32_t groups = WAVE ? BLOCK / kWave : 1;
    auto kern = survey_kernel<LOG_SLOTS, BLOCK, WAVE, META, ENUM, MULTI, FORM, PIECES, WIDE>;
    // attribute and occupancy queries run once per kernel, device and LDS
    // size, so that a survey recorded into a HIP graph issues launches only
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, uint64_t> resident;  // workgroups that fit on the device
    uint64_t fit = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = resident.find({device, L.total});
        if (it != resident.end()) fit = it->second;
    }
    if (!fit) {
        TP_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total));
        int per_cu = 0;
        TP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, L.total));
        if (per_cu < 1) fail(TP_ERR_DEVICE, "survey kernel does not fit on a compute unit");
        int cus = 0;
        TP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
        fit = (uint64_t)per_cu * cus;
        std::lock_guard<std::mutex> lock(mu);
        resident[{device, L.total}] = fit;
    }
    // tiles per claim: as many as keep about 8 claims per claiming wave or
    // workgroup of a full grid
    SurveyParams Q = P;
    const uint64_t units = fit * groups;
    uint32_t claim = WAVE ? kMaxClaimWave : kMaxClaimGroup;
    while (claim > 1 && Q.n_tiles < (uint64_t)claim * units * 8) claim >>= 1;
    Q.claim = claim;
    Q.claim_seg_log = P.rank_gid ? 3u : 0u;  // segments per XCD for batches (kClaimSegs)
    const uint64_t claims = (Q.n_tiles + (uint64_t)claim * groups - 1) / ((uint64_t)claim * groups);
    uint64_t grid = fit;
    if (P.grid_eighths > 0 && P.grid_eighths < 8) grid = std::max<uint64_t>(1, fit * P.grid_eighths / 8);
    if (grid > claims) grid = claims;
    zero_u64<<<1, 64, 0, s>>>(Q.tile_counter, kClaimSegs);
    TP_CHECK_LAUNCH();
    kern<<<(unsigned)grid, BLOCK, L.total, s>>>(Q);
    TP_CHECK_LAUNCH();
}

// Launch a class kernel: with the doubled hit ring where the outputs'
// counters leave LDS for it, else with the plain ring, whose size every LDS
// decision before the launch assumes (counter copies, which kernels fit).
template <int LOG_SLOTS, int BLOCK, bool WAVE, bool META, bool ENUM, bool MULTI, int FORM, bool PIECES = false>
void launch_class(const SurveyParams &P, hipStream_t s, int device)
{
    if (P.n_tiles == 0) return;
    constexpr uint32_t groups = WAVE ? BLOCK / kWave : 1;
    const uint32_t slots = LOG_SLOTS > 0 ? (2u << LOG_SLOTS) + kStash : 0u;
    const uint32_t nc = counter_words<MULTI, FORM>(P);
    auto layout = [&](uint32_t ring) {
        return lds_layout(slots * groups, META || ENUM, nc * groups, BLOCK / kWave, P.lut_shift, FORM == kFormPart,
                          FORM == kFormExt && P.dir_words, ENUM, FORM == kFormExt && (P.outputs & TP_OUT_DEGREE_TABLE),
                          ring);
    };
    constexpr uint32_t wide = ring_size<WAVE, BLOCK, META, ENUM, MULTI, FORM, true>();
    if constexpr (wide > kRing) {
        const LdsLayout L = layout(wide);
        if (L.total <= kLdsLimit) {
            launch_kernel<LOG_SLOTS, BLOCK, WAVE, META, ENUM, MULTI, FORM, PIECES, true>(P, L, s, device);
            return;
        }
    }
    const LdsLayout L = layout(kRing);
    if (L.total > kLdsLimit)
        fail(TP_ERR_UNSUPPORTED, "tripoll_survey: the requested outputs need more LDS than a workgroup may hold");
    launch_kernel<LOG_SLOTS, BLOCK, WAVE, META, ENUM, MULTI, FORM, PIECES, false>(P, L, s, device);
}

// The search variant class c runs with under `strategy`.
uint32_t resolve_variant(const tp_graph *g, int c, uint32_t strategy)
{
    if (strategy == TP_STRAT_GLOBAL_SEARCH) return TP_VAR_SEARCH;
    const uint32_t v = g->plan.variant[c];
    if (v != TP_VAR_DEFAULT) return v;
    if (c == kClassTiny) return TP_VAR_WAVE_TABLE;
    return TP_VAR_GROUP_TABLE;
}

template <bool META, bool ENUM, bool MULTI = false, int FORM = kFormSurvey>
void launch_variant(int c, uint32_t v, const SurveyParams &P0, hipStream_t s, int device)
{
    // as many counter copies as the class's tables leave LDS for; a batch
    // keeps one copy, since its workgroups merge their counters at every
    // change of graph
    SurveyParams P = P0;
    if (c == kClassHuge) {
        // huge targets: tiles over the records cut to each piece
        P.inkey = P.piece_key;
        P.inpay = P.piece_pay;
    }
    if (!P.rank_gid) {
        const uint32_t log_slots = v == TP_VAR_WAVE_TABLE ? kTinyLogSlots
                                   : v == TP_VAR_GROUP_TABLE ? (c >= kClassLarge ? kLargeLogSlots : kSmallLogSlots)
                                                             : 0;
        const bool wave = v == TP_VAR_WAVE_TABLE || v == TP_VAR_WAVE_SEARCH;
        uint32_t top = kMaxCopies;
        if (log_slots == kLargeLogSlots) {
            P.copies = kMaxCopiesLarge;
            if (lds_need<kLargeLogSlots, kLargeBlock, false, META, ENUM, MULTI, FORM, true>(P) <= kLdsLimit)
                top = kMaxCopiesLarge;
        }
        for (P.copies = top; P.copies > 1; P.copies /= 2) {
            size_t need = 0;
            if (log_slots == kTinyLogSlots && wave) need = lds_need<kTinyLogSlots, kSmallBlock, true, META, ENUM, MULTI, FORM>(P);
            else if (log_slots == kLargeLogSlots) need = lds_need<kLargeLogSlots, kLargeBlock, false, META, ENUM, MULTI, FORM>(P);
            else if (log_slots == kSmallLogSlots) need = lds_need<kSmallLogSlots, kSmallBlock, false, META, ENUM, MULTI, FORM>(P);
            else if (wave) need = lds_need<0, kSmallBlock, true, META, ENUM, MULTI, FORM>(P);
            else need = lds_need<0, kSmallBlock, false, META, ENUM, MULTI, FORM>(P);
            if (need <= kLdsLimit) break;
        }
    }
    // a table variant whose tables and counters together overflow LDS (large
    // degree tables) searches Adj+(q) in HBM instead
    // (per-wave forms hold counters per wave, so they overflow first)
    const bool wave_search_fits = lds_need<0, kSmallBlock, true, META, ENUM, MULTI, FORM>(P) <= kLdsLimit;
    if (c == kClassHuge) {
        // the kernels that walk pieces: the large tables, or the HBM search
        // by workgroups or by waves
        if (v == TP_VAR_GROUP_TABLE && lds_need<kLargeLogSlots, kLargeBlock, false, META, ENUM, MULTI, FORM>(P) <= kLdsLimit)
            launch_class<kLargeLogSlots, kLargeBlock, false, META, ENUM, MULTI, FORM, true>(P, s, device);
        else if (v == TP_VAR_WAVE_SEARCH && wave_search_fits)
            launch_class<0, kSmallBlock, true, META, ENUM, MULTI, FORM, true>(P, s, device);
        else
            launch_class<0, kSmallBlock, false, META, ENUM, MULTI, FORM, true>(P, s, device);
        return;
    }
    switch (v) {
    case TP_VAR_WAVE_TABLE:
        if (lds_need<kTinyLogSlots, kSmallBlock, true, META, ENUM, MULTI, FORM>(P) <= kLdsLimit)
            launch_class<kTinyLogSlots, kSmallBlock, true, META, ENUM, MULTI, FORM>(P, s, device);
        else if (wave_search_fits)
            launch_class<0, kSmallBlock, true, META, ENUM, MULTI, FORM>(P, s, device);
        else
            launch_class<0, kSmallBlock, false, META, ENUM, MULTI, FORM>(P, s, device);
        break;
    case TP_VAR_GROUP_TABLE:
        if (c == kClassLarge && lds_need<kLargeLogSlots, kLargeBlock, false, META, ENUM, MULTI, FORM>(P) <= kLdsLimit)
            launch_class<kLargeLogSlots, kLargeBlock, false, META, ENUM, MULTI, FORM>(P, s, device);
        else if (c != kClassLarge && lds_need<kSmallLogSlots, kSmallBlock, false, META, ENUM, MULTI, FORM>(P) <= kLdsLimit)
            launch_class<kSmallLogSlots, kSmallBlock, false, META, ENUM, MULTI, FORM>(P, s, device);
        else
            launch_class<0, kSmallBlock, false, META, ENUM, MULTI, FORM>(P, s, device);
        break;
    case TP_VAR_WAVE_SEARCH:
        if (wave_search_fits)
            launch_class<0, kSmallBlock, true, META, ENUM, MULTI, FORM>(P, s, device);
        else
            launch_class<0, kSmallBlock, false, META, ENUM, MULTI, FORM>(P, s, device);
        break;
    default:
        launch_class<0, kSmallBlock, false, META, ENUM, MULTI, FORM>(P, s, device);
        break;
    }
}

// Launch the target classes in turn.  `timers`, when given, holds one
// EventTimer per class around its launch.
template <bool META, bool ENUM, int FORM = kFormSurvey>
void launch_all(const tp_graph *g, SurveyParams P, uint32_t strategy, hipStream_t s, EventTimer *timers = nullptr)
{
    for (int c = 0; c < kNumClasses; ++c) {
        P.tiles = g->tiles[c].get();
        P.n_tiles = g->n_tiles[c];
        if (timers) timers[c].start();
        launch_variant<META, ENUM, false, FORM>(c, resolve_variant(g, c, strategy), P, s, g->device);
        if (timers) timers[c].stop();
        if (P.class_tri) {
            k_copy_word<<<1, 64, 0, s>>>(P.out + P.o_tri, P.class_tri + c);
            TP_CHECK_LAUNCH();
        }
    }
}

// per_graph: a batch survey (results per graph of a batch)
void validate_spec(const tp_graph *g, const tp_survey_spec *sp, bool per_graph = false)
{
    if (!g || !sp) fail(TP_ERR_INVALID, "tripoll_survey: NULL argument");
    const uint32_t known = TP_OUT_COUNT | TP_OUT_CLOSE_HIST | TP_OUT_LABEL_TABLE | TP_OUT_SPREAD_COUNT |
                           TP_OUT_OPEN_CLOSE | TP_OUT_MAX_EDGE | TP_OUT_DEGREE_TABLE | TP_OUT_DIRECTED;
    if (sp->outputs & ~known) fail(TP_ERR_INVALID, "tripoll_survey: unknown output bits");
    if (sp->reserved != 0) fail(TP_ERR_INVALID, "tripoll_survey: reserved field must be 0");
    if ((sp->outputs & TP_OUT_MAX_EDGE) && sp->max_edge_shift > 31)
        fail(TP_ERR_INVALID, "tripoll_survey: max_edge_shift must be in 0..31");
    if ((sp->outputs & TP_OUT_DEGREE_TABLE) && g->n_graphs && !per_graph)
        fail(TP_ERR_UNSUPPORTED, "tripoll_survey: the degree table of a batch is produced per graph, by "
                                 "tripoll_survey_batch");
    if ((sp->outputs & TP_OUT_DIRECTED) && !g->directed)
        fail(TP_ERR_INVALID, "tripoll_survey: the directed census needs a graph built with TP_EDGES_DIRECTED");
    if (sp->filters & ~(TP_FILT_WINDOW | TP_FILT_LABEL_MASK)) fail(TP_ERR_INVALID, "tripoll_survey: unknown filter bits");
    if (sp->strategy > TP_STRAT_TABLE_STRESS) fail(TP_ERR_INVALID, "tripoll_survey: unknown strategy");
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

// Type of a triangle p <+ q <+ r in the triad census, from the direction
// bits of its three oriented edges (bit 0: an arc from the lower rank, bit 1:
// one towards it): by the number of arcs, then by in- and out-degrees.
// 7 (no counter) when an edge has no direction.
uint8_t directed_type(uint32_t dpq, uint32_t dpr, uint32_t dqr)
{
    if (!dpq || !dpr || !dqr) return 7;
    int out[3] = {0, 0, 0}, in[3] = {0, 0, 0}, arcs = 0;
    auto add = [&](uint32_t d, int a, int b) {
        if (d & 1u) { ++out[a]; ++in[b]; ++arcs; }
        if (d & 2u) { ++out[b]; ++in[a]; ++arcs; }
    };
    add(dpq, 0, 1);
    add(dpr, 0, 2);
    add(dqr, 1, 2);
    if (arcs == 3) return (out[0] == 1 && out[1] == 1 && out[2] == 1) ? 1 : 0;  // 030C, else 030T
    if (arcs == 4) {
        for (int v = 0; v < 3; ++v)
            if (in[v] == 0) return 2;   // 120D: one vertex sends both its arcs
        for (int v = 0; v < 3; ++v)
            if (out[v] == 0) return 3;  // 120U: one vertex receives both
        return 4;                       // 120C
    }
    return arcs == 5 ? 5 : 6;           // 210, 300
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
    P.inkey = g->inkey.get();
    P.inpay = g->inpay.get();
    P.piece_key = g->piece_key.get();
    P.piece_pay = g->piece_pay.get();
    P.kbits = g->kbits;
    P.tile_counter = counter;
    P.out = out;
    P.rank_gid = nullptr;
    P.g_stride = 0;
    P.o_tri = TP_RW_TRIANGLES;
    P.o_spread = TP_RW_SPREAD;
    P.o_probes = TP_RW_PROBES;
    P.o_hist = TP_RW_HIST;
    P.o_table = TP_RW_TABLE;
    P.o_oc = TP_RW_OPEN_CLOSE;
    P.o_maxe = TP_RW_MAX_EDGE;
    P.o_deg = TP_RW_DEGREE;
    P.outputs = sp->outputs | TP_OUT_COUNT;
    P.filters = sp->filters;
    P.table_words = (sp->outputs & TP_OUT_LABEL_TABLE) ? table_size(sp->n_labels) : 0;
    P.oc_words = (sp->outputs & TP_OUT_OPEN_CLOSE) ? 1024 : 0;
    P.maxe_words = (sp->outputs & TP_OUT_MAX_EDGE) ? TP_MAX_EDGE_BINS : 0;
    P.max_edge_shift = sp->max_edge_shift;
    P.copies = 1;  // raised per launch where LDS allows
    // the degree table needs only the bins up to bin(d_max)
    P.deg_words = (sp->outputs & TP_OUT_DEGREE_TABLE) ? table_size(g->dbin_values) : 0;
    P.dbin_rank = g->dbin_rank.get();
    P.dbin_slot = g->dbin_slot.get();
    P.dir_words = ((sp->outputs & TP_OUT_DIRECTED) && g->directed) ? 8u : 0u;
    P.o_dir = TP_RW_DIRECTED;
    P.edir = g->edir.get();
    for (uint32_t i = 0; i < 64; ++i) P.dir_type[i] = directed_type(i >> 4, (i >> 2) & 3u, i & 3u);
    // close < spread_lt  <=>  close <= spread_lt - 1 (close is a uint32)
    P.spread_any = sp->spread_lt > 0;
    P.spread_le = sp->spread_lt == 0 ? 0u : (uint32_t)std::min<uint64_t>(sp->spread_lt - 1, 0xffffffffull);
    // window bounds beyond the uint32 time range clamp to it; an empty clamped
    // window (t_lo > 2^32 - 1) keeps nothing
    P.t_lo32 = (uint32_t)std::min<uint64_t>(sp->t_lo, 0xffffffffull);
    P.t_hi32 = (uint32_t)std::min<uint64_t>(sp->t_hi, 0xffffffffull);
    P.window_empty = sp->t_lo > 0xffffffffull;
    // the table-stress strategy allows a single placement attempt, so that
    // the stash and the HBM fallback are exercised
    P.max_kicks = sp->strategy == TP_STRAT_TABLE_STRESS ? 1u : kMaxKicks;
    P.lut_shift = 0;
    if ((sp->outputs & TP_OUT_LABEL_TABLE) || (sp->filters & TP_FILT_LABEL_MASK))
        while ((1u << P.lut_shift) < sp->n_labels) ++P.lut_shift;
    for (int i = 0; i < 13; ++i) P.label_mask[i] = sp->label_mask[i];
    P.perm = g->perm.get();
    P.n = g->n;
    return P;
}

bool needs_meta(const tp_survey_spec *sp)
{
    return (sp->outputs & ~TP_OUT_COUNT) != 0 || sp->filters != 0;
}

bool needs_ext(const tp_survey_spec *sp)
{
    return (sp->outputs & (TP_OUT_MAX_EDGE | TP_OUT_DEGREE_TABLE | TP_OUT_DIRECTED)) != 0;
}

// Enqueue a whole survey into the caller's result buffer (which also holds
// the tile counter).  Allocates nothing.
template <bool ENUM>
void survey_enqueue(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *dev_out, hipStream_t s,
                    uint32_t *enum_out = nullptr, uint64_t enum_cap = 0, EventTimer *timers = nullptr,
                    const uint32_t *enum_srow = nullptr)
{
    zero_u64<<<grid_for(TP_RESULT_WORDS, 256), 256, 0, s>>>(dev_out, TP_RESULT_WORDS);
    TP_CHECK_LAUNCH();
    SurveyParams P = make_params(g, sp, dev_out, dev_out + kRwClaim);
    if (g->m == 0 || g->n_in == 0) return;
    if (!ENUM) P.class_tri = dev_out + TP_RW_CLASS_TRI;
    if (ENUM) {
        P.enum_out = enum_out;
        P.enum_cap = enum_cap;
        P.enum_count = dev_out + TP_RW_SCRATCH + 1;
        P.enum_srow = enum_srow;
        launch_all<true, true>(g, P, TP_STRAT_AUTO, s);
    } else if (needs_ext(sp)) {
        launch_all<true, false, kFormExt>(g, P, sp->strategy, s, timers);
    } else if (needs_meta(sp)) {
        launch_all<true, false>(g, P, sp->strategy, s, timers);
    } else {
        launch_all<false, false>(g, P, sp->strategy, s, timers);
    }
}

uint32_t batch_words(const tp_survey_spec *sp)
{
    uint32_t w = TP_BW_TABLE;
    if (sp->outputs & TP_OUT_LABEL_TABLE) w += table_size(sp->n_labels);
    if (sp->outputs & TP_OUT_OPEN_CLOSE) w += 1024;
    if (sp->outputs & TP_OUT_MAX_EDGE) w += TP_MAX_EDGE_BINS;
    if (sp->outputs & TP_OUT_DEGREE_TABLE) w += TP_DEGREE_MAX;
    if (sp->outputs & TP_OUT_DIRECTED) w += 8;
    return w;
}

uint32_t graph_count(const tp_graph *g) { return g->n_graphs ? g->n_graphs : 1u; }

// Enqueue the survey of every graph of a batch into per-graph blocks of
// `dev_out`, followed by the tile counter.  Allocates nothing.
void survey_batch_enqueue(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *dev_out, hipStream_t s)
{
    const uint32_t words = batch_words(sp);
    const uint64_t total = (uint64_t)graph_count(g) * words + TP_BATCH_SCRATCH_WORDS;
    zero_u64<<<grid_for(total, 256), 256, 0, s>>>(dev_out, total);
    TP_CHECK_LAUNCH();
    SurveyParams P = make_params(g, sp, dev_out, dev_out + (total - kClaimWords));
    P.rank_gid = g->n_graphs ? g->rank_gid.get() : nullptr;
    P.g_stride = words;
    P.o_tri = TP_BW_TRIANGLES;
    P.o_spread = TP_BW_SPREAD;
    P.o_probes = TP_BW_PROBES;
    P.o_hist = TP_BW_HIST;
    P.o_table = TP_BW_TABLE;
    P.o_oc = TP_BW_TABLE + P.table_words;
    P.o_maxe = P.o_oc + P.oc_words;
    P.o_deg = P.o_maxe + P.maxe_words;
    P.o_dir = P.o_deg + ((sp->outputs & TP_OUT_DEGREE_TABLE) ? TP_DEGREE_MAX : 0u);
    if (g->m == 0 || g->n_in == 0) return;
    if (needs_ext(sp))
        launch_all<true, false, kFormExt>(g, P, sp->strategy, s);
    else if (needs_meta(sp))
        launch_all<true, false>(g, P, sp->strategy, s);
    else
        launch_all<false, false>(g, P, sp->strategy, s);
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
    for (uint32_t i = 0; i < TP_MAX_EDGE_BINS; ++i) out->max_edge[i] = h[TP_RW_MAX_EDGE + i];
    for (uint32_t i = 0; i < TP_DEGREE_MAX; ++i) out->degree_table[i] = h[TP_RW_DEGREE + i];
    for (uint32_t i = 0; i < 7; ++i) out->directed[i] = h[TP_RW_DIRECTED + i];
    for (int c = 0; c < kNumClasses; ++c)
        out->class_triangles[c] = h[TP_RW_CLASS_TRI + c] - (c ? h[TP_RW_CLASS_TRI + c - 1] : 0ull);
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
        EventTimer cls[kNumClasses] = {EventTimer(s), EventTimer(s), EventTimer(s), EventTimer(s)};
        all.start();
        kern.start();
        survey_enqueue<false>(g, spec, res.get(), s, nullptr, 0, cls);
        kern.stop();
        std::vector<unsigned long long> h(TP_RESULT_WORDS);
        TP_HIP(hipMemcpyAsync(h.data(), res.get(), TP_RESULT_WORDS * 8, hipMemcpyDeviceToHost, s));
        all.stop();
        TP_HIP(hipStreamSynchronize(s));
        copy_result(h, out);
        out->kernel_ms = kern.ms();
        out->total_ms = all.ms();
        for (int c = 0; c < kNumClasses; ++c) out->class_ms[c] = g->n_tiles[c] ? cls[c].ms() : 0.f;
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

// ---------------------------------------------------------------- exact counting set of Algorithm 3

namespace {

__global__ void k_maxe_flags(const unsigned long long *keys, uint64_t n, uint32_t *occupied)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        occupied[i] = keys[i] != 0ull ? 1u : 0u;
}

// the occupied slots packed in slot order: value (the sort key), its place
// in the packed order, and its count
__global__ void k_maxe_pack(const unsigned long long *keys, const unsigned long long *counts, const uint64_t *pos,
                            uint64_t n, uint64_t *value, uint32_t *place, unsigned long long *count)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = keys[i];
        if (!k) continue;
        const uint64_t j = pos[i];
        value[j] = k - 1ull;
        place[j] = (uint32_t)j;
        count[j] = counts[i];
    }
}

__global__ void k_maxe_out(const uint64_t *value, const uint32_t *place, const unsigned long long *count, uint64_t n,
                           uint32_t *out_value, uint64_t *out_count)
{
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
        out_value[j] = (uint32_t)value[j];
        out_count[j] = count[place[j]];
    }
}

}  // namespace

extern "C" tp_status tripoll_max_edge_counts(const tp_graph *g, const tp_survey_spec *spec, uint32_t *dev_values,
                                             uint64_t *dev_counts, uint64_t capacity, uint64_t *n_values, void *stream)
{
    return guard([&] {
        if (!spec || !n_values) fail(TP_ERR_INVALID, "tripoll_max_edge_counts: NULL argument");
        if (capacity && (!dev_values || !dev_counts))
            fail(TP_ERR_INVALID, "tripoll_max_edge_counts: NULL output buffer");
        *n_values = 0;
        tp_survey_spec sp = *spec;
        sp.outputs = TP_OUT_COUNT;
        sp.max_edge_shift = 0;
        validate_spec(g, &sp);
        if (g->n_graphs) fail(TP_ERR_UNSUPPORTED, "tripoll_max_edge_counts: single graphs only");
        if (g->m == 0 || g->n_in == 0) return;
        hipStream_t s = (hipStream_t)stream;
        // at most m distinct times: a table of at least 2 m slots stays at
        // most half full
        uint64_t slots = 1024;
        while (slots < 2 * g->m && slots < (1ull << 32)) slots <<= 1;
        DArray<unsigned long long> keys(slots, s), counts(slots, s), res(TP_RESULT_WORDS, s), flag(1, s);
        zero_u64<<<grid_for(slots, 256), 256, 0, s>>>(keys.get(), slots);
        zero_u64<<<grid_for(slots, 256), 256, 0, s>>>(counts.get(), slots);
        zero_u64<<<grid_for(TP_RESULT_WORDS, 256), 256, 0, s>>>(res.get(), TP_RESULT_WORDS);
        zero_u64<<<1, 64, 0, s>>>(flag.get(), 1);
        TP_CHECK_LAUNCH();
        SurveyParams P = make_params(g, &sp, res.get(), res.get() + kRwClaim);
        P.maxe_keys = keys.get();
        P.maxe_counts = counts.get();
        P.maxe_mask = slots - 1;
        P.maxe_overflow = reinterpret_cast<unsigned *>(flag.get());
        launch_all<true, false, kFormExt>(g, P, sp.strategy, s);
        // pack the occupied slots, then sort them by value
        DArray<uint32_t> occupied(slots, s);
        DArray<uint64_t> pos(slots + 1, s);
        k_maxe_flags<<<grid_for(slots, 256), 256, 0, s>>>(keys.get(), slots, occupied.get());
        TP_CHECK_LAUNCH();
        scan_u32_to_u64(occupied.get(), pos.get(), slots, s);
        uint64_t total = 0;
        unsigned long long over = 0;
        TP_HIP(hipMemcpyAsync(&total, pos.get() + slots, 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipMemcpyAsync(&over, flag.get(), 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        if (over) fail(TP_ERR_DEVICE, "tripoll_max_edge_counts: a value found no slot in the table");
        *n_values = total;
        if (total > capacity)
            fail(TP_ERR_INVALID, "tripoll_max_edge_counts: " + std::to_string(total) + " distinct values, capacity " +
                                     std::to_string(capacity));
        if (total == 0) return;
        DArray<uint64_t> va(total, s), vb(total, s);
        DArray<uint32_t> pa(total, s), pb(total, s);
        DArray<unsigned long long> cnt(total, s);
        k_maxe_pack<<<grid_for(slots, 256), 256, 0, s>>>(keys.get(), counts.get(), pos.get(), slots, va.get(), pa.get(),
                                                         cnt.get());
        TP_CHECK_LAUNCH();
        const bool alt = radix_sort_pairs(va.get(), pa.get(), vb.get(), pb.get(), total, 32, s);
        k_maxe_out<<<grid_for(total, 256), 256, 0, s>>>(alt ? vb.get() : va.get(), alt ? pb.get() : pa.get(), cnt.get(),
                                                        total, dev_values, dev_counts);
        TP_CHECK_LAUNCH();
        TP_HIP(hipStreamSynchronize(s));
    });
}

// ---------------------------------------------------------------- survey without allocation
// The result words of tripoll_survey_noalloc live in one file-scope device
// array (each GPU holds its own copy until the process ends) instead of a
// buffer taken from the allocator.  Its name is a host-side stand-in in host
// code: the device address of each GPU's copy comes from
// hipGetSymbolAddress, called once per device with that device current, and
// only that address is handed to kernels and copies.
constexpr size_t kStaticResultWords = TP_RESULT_WORDS;
static __device__ __align__(256) unsigned long long scratch[kStaticResultWords];

namespace {

constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
unsigned long long *g_static_ptr[kMaxStaticDevices] = {};

// Device address of `scratch` on `device`, which must be current.
unsigned long long *static_result_words(int device)
{
    if (device < 0 || device >= kMaxStaticDevices)
        fail(TP_ERR_UNSUPPORTED, "tripoll_survey_noalloc: device index beyond " + std::to_string(kMaxStaticDevices));
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[device]) {
        void *p = nullptr;
        TP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(TP_ERR_DEVICE, "tripoll_survey_noalloc: no device address for the result words");
        g_static_ptr[device] = static_cast<unsigned long long *>(p);
    }
    return g_static_ptr[device];
}

}  // namespace

extern "C" tp_status tripoll_survey_noalloc(const tp_graph *g, const tp_survey_spec *spec, tp_survey_result *out,
                                            void *stream)
{
    static_assert(TP_RESULT_WORDS <= kStaticResultWords, "the static result words hold a whole result");
    static_assert(offsetof(tp_survey_result, directed) == TP_RW_DIRECTED * 8,
                  "the result struct starts with the device result words");
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_survey_noalloc: NULL result");
        validate_spec(g, spec);
        int dev = 0;
        TP_HIP(hipGetDevice(&dev));
        if (dev != g->device) fail(TP_ERR_INVALID, "tripoll_survey_noalloc: the graph's device must be current");
        unsigned long long *words = static_result_words(dev);
        hipStream_t s = (hipStream_t)stream;
        // survey_enqueue clears the words with a fill kernel, then surveys
        survey_enqueue<false>(g, spec, words, s);
        unsigned long long snap[kNumClasses];
        TP_HIP(hipMemcpyAsync(out, words, TP_RW_SCRATCH * 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipMemcpyAsync(snap, words + TP_RW_CLASS_TRI, sizeof(snap), hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        out->directed[7] = 0;
        out->kernel_ms = 0.f;
        out->total_ms = 0.f;
        for (int c = 0; c < kNumClasses; ++c) {
            out->class_ms[c] = 0.f;
            out->class_triangles[c] = snap[c] - (c ? snap[c - 1] : 0ull);
        }
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
        DArray<uint32_t> srow;
        slot_rows(g, srow, s);
        survey_enqueue<true>(g, &sp, res.get(), s, dev_records, capacity, nullptr, srow.get());
        unsigned long long found = 0;
        TP_HIP(hipMemcpyAsync(&found, res.get() + TP_RW_TRIANGLES, 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        *n_found = found;
    });
}

struct tp_enum_stream {
    const tp_graph *g = nullptr;
    tp_survey_spec spec{};
    uint64_t n_tiles = 0, next = 0, total = 0, max_tile = 0, emitted = 0;
    uint64_t class_first[kNumClasses + 1] = {};  // first global tile of each class
    DArray<uint64_t> base;       // [n_tiles + 1] first record of each tile
    DArray<unsigned> cursor;     // [n_tiles] records written per tile
    DArray<unsigned long long> res;
    DArray<uint64_t> chunk;      // [3] result of k_enum_chunk
    DArray<uint32_t> srow;       // [m] pivot of every CSR slot
};

namespace {

// Launch the enumeration form over global tiles [t0, t1), class by class.
void enum_tiles(tp_enum_stream *e, SurveyParams P, uint64_t t0, uint64_t t1, hipStream_t s)
{
    const tp_graph *g = e->g;
    for (int c = 0; c < kNumClasses; ++c) {
        const uint64_t lo = std::max(t0, e->class_first[c]), hi = std::min(t1, e->class_first[c + 1]);
        if (lo >= hi) continue;
        P.tiles = g->tiles[c].get() + (lo - e->class_first[c]);
        P.n_tiles = hi - lo;
        P.tile_gbase = lo;
        launch_variant<true, true>(c, resolve_variant(g, c, TP_STRAT_AUTO), P, s, g->device);
    }
}

}  // namespace

extern "C" tp_status tripoll_enum_open(const tp_graph *g, const tp_survey_spec *spec, void *stream,
                                       tp_enum_stream **out, uint64_t *total, uint64_t *max_tile)
{
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_enum_open: NULL output");
        validate_spec(g, spec);
        hipStream_t s = (hipStream_t)stream;
        auto e = std::make_unique<tp_enum_stream>();
        e->g = g;
        e->spec = *spec;
        e->spec.outputs = TP_OUT_COUNT;
        for (int c = 0; c < kNumClasses; ++c) e->class_first[c + 1] = e->class_first[c] + g->n_tiles[c];
        e->n_tiles = e->class_first[kNumClasses];
        const uint64_t T = e->n_tiles;
        e->base.reset(T + 1, s);
        e->cursor.reset(std::max<uint64_t>(T, 1), s);
        e->res.reset(TP_RESULT_WORDS, s);
        e->chunk.reset(3, s);
        slot_rows(g, e->srow, s);
        DArray<unsigned> count(std::max<uint64_t>(T, 1), s);
        zero_u64<<<grid_for(TP_RESULT_WORDS, 256), 256, 0, s>>>(e->res.get(), TP_RESULT_WORDS);
        TP_CHECK_LAUNCH();
        TP_HIP(hipMemsetAsync(count.get(), 0, std::max<uint64_t>(T, 1) * sizeof(unsigned), s));
        TP_HIP(hipMemsetAsync(e->cursor.get(), 0, std::max<uint64_t>(T, 1) * sizeof(unsigned), s));
        if (T && g->m && g->n_in) {
            // one counting pass: the records of every tile
            SurveyParams P = make_params(g, &e->spec, e->res.get(), e->res.get() + kRwClaim);
            P.enum_tile_count = count.get();
            P.enum_srow = e->srow.get();
            enum_tiles(e.get(), P, 0, T, s);
        }
        if (T) scan_u32_to_u64(count.get(), e->base.get(), T, s);
        else TP_HIP(hipMemsetAsync(e->base.get(), 0, sizeof(uint64_t), s));
        unsigned long long *mx = e->res.get() + TP_RW_SCRATCH + 2;
        zero_u64<<<1, 64, 0, s>>>(mx, 1);
        TP_CHECK_LAUNCH();
        if (T) {
            k_max_u32<<<grid_for(T, 256), 256, 0, s>>>(count.get(), T, mx);
            TP_CHECK_LAUNCH();
        }
        uint64_t h[2] = {0, 0};
        TP_HIP(hipMemcpyAsync(&h[0], e->base.get() + T, 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipMemcpyAsync(&h[1], mx, 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        e->total = h[0];
        e->max_tile = h[1];
        if (total) *total = e->total;
        if (max_tile) *max_tile = e->max_tile;
        *out = e.release();
    });
}

extern "C" tp_status tripoll_enum_next(tp_enum_stream *e, uint32_t *dev_records, uint64_t capacity,
                                       uint64_t *n_written, void *stream)
{
    return guard([&] {
        if (!e || !n_written || (capacity && !dev_records)) fail(TP_ERR_INVALID, "tripoll_enum_next: bad argument");
        hipStream_t s = (hipStream_t)stream;
        *n_written = 0;
        // skip tiles without records, then take as many whole tiles as fit
        if (e->next >= e->n_tiles || e->emitted == e->total) {
            e->next = e->n_tiles;
            return;
        }
        k_enum_chunk<<<1, 64, 0, s>>>(e->base.get(), e->n_tiles, e->next, capacity, e->chunk.get());
        TP_CHECK_LAUNCH();
        uint64_t c[3];
        TP_HIP(hipMemcpyAsync(c, e->chunk.get(), sizeof(c), hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        uint64_t t1 = c[0];
        if (c[2] == c[1]) {
            // only empty tiles fit before the first that does not: move past them
            e->next = t1;
            if (e->next >= e->n_tiles) return;
            k_enum_chunk<<<1, 64, 0, s>>>(e->base.get(), e->n_tiles, e->next, capacity, e->chunk.get());
            TP_CHECK_LAUNCH();
            TP_HIP(hipMemcpyAsync(c, e->chunk.get(), sizeof(c), hipMemcpyDeviceToHost, s));
            TP_HIP(hipStreamSynchronize(s));
            t1 = c[0];
        }
        if (t1 == e->next)
            fail(TP_ERR_INVALID, "tripoll_enum_next: capacity " + std::to_string(capacity) +
                                     " is below the next tile's records (the largest tile has " +
                                     std::to_string(e->max_tile) + ")");
        SurveyParams P = make_params(e->g, &e->spec, e->res.get(), e->res.get() + kRwClaim);
        P.enum_out = dev_records;
        P.enum_cap = capacity;
        P.enum_tile_base = e->base.get();
        P.enum_tile_cursor = e->cursor.get();
        P.enum_srow = e->srow.get();
        P.enum_chunk_base = c[1];
        enum_tiles(e, P, e->next, t1, s);
        TP_HIP(hipStreamSynchronize(s));
        *n_written = c[2] - c[1];
        e->emitted += *n_written;
        e->next = t1;
    });
}

extern "C" tp_status tripoll_enum_close(tp_enum_stream *e)
{
    return guard([&] { delete e; });
}

extern "C" tp_status tripoll_participation(const tp_graph *g, const tp_survey_spec *spec, uint64_t *vertex_counts,
                                           uint64_t *edge_counts, uint64_t *triangles, void *stream)
{
    return guard([&] {
        validate_spec(g, spec);
        hipStream_t s = (hipStream_t)stream;
        // the filters of the spec apply; its outputs do not.  A batch is
        // counted as the union of its graphs, which no triangle spans: its
        // vertex ids and CSR slots are those of the union, graph by graph
        tp_survey_spec sp = *spec;
        sp.outputs = TP_OUT_COUNT;
        DArray<unsigned long long> res(TP_RESULT_WORDS, s);
        zero_u64<<<grid_for(TP_RESULT_WORDS, 256), 256, 0, s>>>(res.get(), TP_RESULT_WORDS);
        TP_CHECK_LAUNCH();
        DArray<unsigned long long> own;
        unsigned long long *edge = reinterpret_cast<unsigned long long *>(edge_counts);
        if (!edge) {
            own.reset(std::max<uint64_t>(g->m, 1), s);
            edge = own.get();
        }
        if (g->m) {
            zero_u64<<<grid_for(g->m, 256), 256, 0, s>>>(edge, g->m);
            TP_CHECK_LAUNCH();
        }
        SurveyParams P = make_params(g, &sp, res.get(), res.get() + kRwClaim);
        P.part_edge = edge;
        if (g->m && g->n_in) launch_all<true, false, kFormPart>(g, P, sp.strategy, s);
        if (vertex_counts) {
            DArray<unsigned long long> acc(g->n, s);
            zero_u64<<<grid_for(g->n, 256), 256, 0, s>>>(acc.get(), g->n);
            TP_CHECK_LAUNCH();
            k_part_rows<<<grid_for((size_t)g->n * kWave, 256), 256, 0, s>>>(g->rowptr.get(), g->col.get(), g->n, edge,
                                                                           acc.get());
            TP_CHECK_LAUNCH();
            k_part_vertex<<<grid_for(g->n, 256), 256, 0, s>>>(acc.get(), g->perm.get(), g->n, vertex_counts);
            TP_CHECK_LAUNCH();
        }
        unsigned long long tri = 0;
        TP_HIP(hipMemcpyAsync(&tri, res.get() + TP_RW_TRIANGLES, 8, hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        if (triangles) *triangles = tri;
    });
}

extern "C" tp_status tripoll_graph_count(const tp_graph *g, uint32_t *n_graphs)
{
    return guard([&] {
        if (!g || !n_graphs) fail(TP_ERR_INVALID, "tripoll_graph_count: NULL argument");
        *n_graphs = graph_count(g);
    });
}

extern "C" uint64_t tripoll_batch_words(const tp_survey_spec *spec)
{
    return spec ? batch_words(spec) : 0;
}

extern "C" tp_status tripoll_survey_batch(const tp_graph *g, const tp_survey_spec *spec, uint64_t *dev_out,
                                          void *stream)
{
    return guard([&] {
        if (!dev_out) fail(TP_ERR_INVALID, "tripoll_survey_batch: NULL output");
        validate_spec(g, spec, true);
        survey_batch_enqueue(g, spec, reinterpret_cast<unsigned long long *>(dev_out), (hipStream_t)stream);
    });
}

// ================================================================ recorded launches

struct tp_launch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~tp_launch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

extern "C" tp_status tripoll_survey_capture(const tp_graph *g, const tp_survey_spec *spec, uint64_t *dev_out,
                                            tp_launch **out)
{
    return guard([&] {
        if (!dev_out || !out) fail(TP_ERR_INVALID, "tripoll_survey_capture: NULL argument");
        validate_spec(g, spec, true);
        // the kernels' attributes are set outside the capture: one eager
        // survey on a private stream prepares every launch.  It writes a
        // temporary buffer of the same size, never dev_out, which work on
        // the caller's streams may still be using.
        hipStream_t cs = nullptr;
        TP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        struct StreamGuard {
            hipStream_t s;
            ~StreamGuard() { (void)hipStreamDestroy(s); }
        } sg{cs};
        {
            const uint64_t words = (uint64_t)graph_count(g) * batch_words(spec) + TP_BATCH_SCRATCH_WORDS;
            DArray<unsigned long long> prep(words, cs);
            survey_batch_enqueue(g, spec, prep.get(), cs);
            TP_HIP(hipStreamSynchronize(cs));
        }
        auto L = std::make_unique<tp_launch>();
        TP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            survey_batch_enqueue(g, spec, reinterpret_cast<unsigned long long *>(dev_out), cs);
        } catch (...) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(cs, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            throw;
        }
        TP_HIP(hipStreamEndCapture(cs, &L->graph));
        TP_HIP(hipGraphInstantiate(&L->exec, L->graph, nullptr, nullptr, 0));
        *out = L.release();
    });
}

extern "C" tp_status tripoll_launch_replay(tp_launch *launch, void *stream)
{
    return guard([&] {
        if (!launch) fail(TP_ERR_INVALID, "tripoll_launch_replay: NULL launch");
        TP_HIP(hipGraphLaunch(launch->exec, (hipStream_t)stream));
    });
}

extern "C" tp_status tripoll_launch_free(tp_launch *launch)
{
    return guard([&] { delete launch; });
}

// ================================================================ multi-request passes

SlotSpec tp::make_slot(const tp_survey_spec &sp)
{
    SlotSpec S{};
    S.outputs = sp.outputs | TP_OUT_COUNT;
    S.filters = sp.filters;
    S.t_lo = (uint32_t)std::min<uint64_t>(sp.t_lo, 0xffffffffull);
    S.t_hi = (uint32_t)std::min<uint64_t>(sp.t_hi, 0xffffffffull);
    S.window_empty = sp.t_lo > 0xffffffffull;
    S.spread_any = sp.spread_lt > 0;
    S.spread_le = sp.spread_lt == 0 ? 0u : (uint32_t)std::min<uint64_t>(sp.spread_lt - 1, 0xffffffffull);
    S.off = 0;
    for (int i = 0; i < 13; ++i) S.label_mask[i] = sp.label_mask[i];
    return S;
}

uint32_t tp::slot_words(uint32_t n_labels) { return TP_BW_TABLE + table_size(n_labels); }

void tp::zero_words(unsigned long long *p, size_t n, hipStream_t s)
{
    if (!n) return;
    zero_u64<<<grid_for(n, 256), 256, 0, s>>>(p, n);
    TP_CHECK_LAUNCH();
}

void tp::multi_segment_enqueue(const tp_graph *g, const SlotSpec *dev_slots, uint32_t n_slots, uint32_t n_labels,
                               bool labels, unsigned long long *dev_out, unsigned long long *dev_counter, uint32_t seg,
                               uint32_t n_seg, uint32_t grid_eighths, hipStream_t s)
{
    if (n_slots == 0 || n_slots > kMaxSlots) fail(TP_ERR_INVALID, "multi-request pass: 1..16 slots");
    if (n_seg == 0 || seg >= n_seg) fail(TP_ERR_INVALID, "multi-request pass: bad segment");
    if (g->m == 0 || g->n_in == 0) return;
    tp_survey_spec sp{};
    sp.outputs = TP_OUT_COUNT | TP_OUT_CLOSE_HIST;
    sp.n_labels = n_labels;
    SurveyParams P = make_params(g, &sp, dev_out, dev_counter);
    P.slots = dev_slots;
    P.n_slots = n_slots;
    P.slot_words = slot_words(n_labels);
    P.g_stride = P.slot_words;
    P.slot_labels = labels ? 1u : 0u;
    P.lut_shift = 0;
    if (labels)
        while ((1u << P.lut_shift) < n_labels) ++P.lut_shift;
    P.grid_eighths = grid_eighths;
    for (int c = 0; c < kNumClasses; ++c) {
        const uint64_t nt = g->n_tiles[c];
        const uint64_t a = nt * seg / n_seg, b = nt * (seg + 1) / n_seg;
        if (a == b) continue;
        // the kernel walks its tile list from the end
        P.tiles = g->tiles[c].get() + a;
        P.n_tiles = b - a;
        launch_variant<true, false, true>(c, resolve_variant(g, c, TP_STRAT_AUTO), P, s, g->device);
    }
}

void tp::solo_segment_enqueue(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *dev_out, uint32_t seg,
                              uint32_t n_seg, uint32_t grid_eighths, hipStream_t s)
{
    if (n_seg == 0 || seg >= n_seg) fail(TP_ERR_INVALID, "single-request segment: bad segment");
    validate_spec(g, sp);
    if (g->m == 0 || g->n_in == 0) return;
    SurveyParams P = make_params(g, sp, dev_out, dev_out + kRwClaim);
    P.grid_eighths = grid_eighths;
    for (int c = 0; c < kNumClasses; ++c) {
        const uint64_t nt = g->n_tiles[c];
        const uint64_t a = nt * seg / n_seg, b = nt * (seg + 1) / n_seg;
        if (a == b) continue;
        P.tiles = g->tiles[c].get() + a;
        P.n_tiles = b - a;
        const uint32_t v = resolve_variant(g, c, sp->strategy);
        if (needs_ext(sp)) launch_variant<true, false, false, kFormExt>(c, v, P, s, g->device);
        else if (needs_meta(sp)) launch_variant<true, false>(c, v, P, s, g->device);
        else launch_variant<false, false>(c, v, P, s, g->device);
    }
}

// ================================================================ plan and tuning

namespace {

bool variant_allowed(int c, uint32_t v)
{
    switch (v) {
    case TP_VAR_DEFAULT:
    case TP_VAR_SEARCH:
    case TP_VAR_WAVE_SEARCH:
        return true;
    case TP_VAR_WAVE_TABLE:
        return c == kClassTiny;
    case TP_VAR_GROUP_TABLE:
        return true;
    default:
        return false;
    }
}

void check_plan(const tp_plan *p)
{
    for (int c = 0; c < kNumClasses; ++c) {
        if (!variant_allowed(c, p->variant[c]))
            fail(TP_ERR_INVALID, "tripoll_set_plan: variant " + std::to_string(p->variant[c]) +
                                     " cannot serve class " + std::to_string(c));
        const uint32_t r = p->tile_records[c];
        if (r < 16 || r > 65536 || (r & (r - 1)))
            fail(TP_ERR_INVALID, "tripoll_set_plan: tile_records must be a power of two in [16, 65536]");
    }
}

PlanCfg to_cfg(const tp_plan *p)
{
    PlanCfg c{};
    for (int i = 0; i < kNumClasses; ++i) {
        c.variant[i] = p->variant[i];
        c.tile_records[i] = p->tile_records[i];
    }
    return c;
}

// Device time of class c's launch under variant v, on the graph's current
// tiles.  `reps` launches; the fastest counts.
float time_class(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *buf, int c, uint32_t v, int reps,
                 hipStream_t s)
{
    SurveyParams P = make_params(g, sp, buf, buf + kRwClaim);
    P.tiles = g->tiles[c].get();
    P.n_tiles = g->n_tiles[c];
    float best = 0.f;
    for (int r = 0; r < reps; ++r) {
        EventTimer t(s);
        t.start();
        if (needs_ext(sp))
            launch_variant<true, false, false, kFormExt>(c, v, P, s, g->device);
        else if (needs_meta(sp))
            launch_variant<true, false>(c, v, P, s, g->device);
        else
            launch_variant<false, false>(c, v, P, s, g->device);
        t.stop();
        const float ms = t.ms();
        if (r == 0 || ms < best) best = ms;
    }
    return best;
}

}  // namespace

extern "C" tp_status tripoll_get_plan(const tp_graph *g, tp_plan *out)
{
    return guard([&] {
        if (!g || !out) fail(TP_ERR_INVALID, "tripoll_get_plan: NULL argument");
        for (int c = 0; c < kNumClasses; ++c) {
            out->variant[c] = g->plan.variant[c];
            out->tile_records[c] = g->plan.tile_records[c];
        }
    });
}

extern "C" tp_status tripoll_set_plan(tp_graph *g, const tp_plan *plan, void *stream)
{
    return guard([&] {
        if (!g || !plan) fail(TP_ERR_INVALID, "tripoll_set_plan: NULL argument");
        check_plan(plan);
        plan_graph(g, to_cfg(plan), (hipStream_t)stream);
        g->stats.device_bytes = graph_bytes(g);
    });
}

extern "C" tp_status tripoll_tune(tp_graph *g, const tp_survey_spec *spec, void *stream, tp_tune_result *out)
{
    return guard([&] {
        if (!out) fail(TP_ERR_INVALID, "tripoll_tune: NULL result");
        validate_spec(g, spec);
        hipStream_t s = (hipStream_t)stream;
        tp_survey_spec sp = *spec;
        sp.strategy = TP_STRAT_AUTO;
        DArray<unsigned long long> buf(TP_RESULT_WORDS, s);
        zero_u64<<<grid_for(TP_RESULT_WORDS, 256), 256, 0, s>>>(buf.get(), TP_RESULT_WORDS);
        TP_CHECK_LAUNCH();
        static const uint32_t kCaps[] = {256, 1024, 4096, 16384};
        static const std::vector<uint32_t> kCands[kNumClasses] = {
            {TP_VAR_WAVE_TABLE, TP_VAR_GROUP_TABLE, TP_VAR_WAVE_SEARCH},
            {TP_VAR_GROUP_TABLE, TP_VAR_SEARCH, TP_VAR_WAVE_SEARCH},
            {TP_VAR_GROUP_TABLE, TP_VAR_SEARCH},
            {TP_VAR_GROUP_TABLE, TP_VAR_SEARCH}};
        tp_tune_result r{};
        float best[kNumClasses];
        uint32_t best_v[kNumClasses], best_cap[kNumClasses];
        for (int c = 0; c < kNumClasses; ++c) {
            best[c] = -1.f;
            best_v[c] = TP_VAR_DEFAULT;
            best_cap[c] = default_tile_records(c);
        }
        for (uint32_t cap : kCaps) {
            PlanCfg cfg{};
            for (int c = 0; c < kNumClasses; ++c) cfg.tile_records[c] = cap;
            plan_graph(g, cfg, s);
            for (int c = 0; c < kNumClasses; ++c) {
                if (g->n_tiles[c] == 0) continue;
                const uint32_t dflt = resolve_variant(g, c, TP_STRAT_AUTO);
                for (uint32_t v : kCands[c]) {
                    // a warm-up launch, then the faster of two timed ones
                    (void)time_class(g, &sp, buf.get(), c, v, 1, s);
                    const float ms = time_class(g, &sp, buf.get(), c, v, 2, s);
                    ++r.trials;
                    if (cap == default_tile_records(c) && v == dflt) r.default_ms[c] = ms;
                    if (best[c] < 0.f || ms < best[c]) {
                        best[c] = ms;
                        best_v[c] = v;
                        best_cap[c] = cap;
                    }
                }
            }
        }
        // keep the default unless the best is clearly faster
        PlanCfg fin{};
        for (int c = 0; c < kNumClasses; ++c) {
            fin.variant[c] = TP_VAR_DEFAULT;
            fin.tile_records[c] = default_tile_records(c);
            if (best[c] >= 0.f && best[c] < 0.97f * r.default_ms[c]) {
                fin.variant[c] = best_v[c];
                fin.tile_records[c] = best_cap[c];
            }
        }
        plan_graph(g, fin, s);
        g->stats.device_bytes = graph_bytes(g);
        for (int c = 0; c < kNumClasses; ++c) {
            r.chosen.variant[c] = fin.variant[c];
            r.chosen.tile_records[c] = fin.tile_records[c];
            r.tuned_ms[c] = g->n_tiles[c] ? time_class(g, &sp, buf.get(), c, resolve_variant(g, c, TP_STRAT_AUTO), 2, s)
                                          : 0.f;
        }
        TP_HIP(hipStreamSynchronize(s));
        *out = r;
    });
}
