// build.hip -- graph builder: raw edge list -> degree-ordered directed graph
// with co-located metadata, its in-edge index and the survey's tile plan.
//
// Phases (all device-resident after the upload):
//   0 canonicalise: (u,v,t) -> key (min<<b | max), self-loops to a sentinel
//   1 radix sort of (key, t)
//   2 dedup: one edge per pair with the minimum time (the chronologically
//     first copy, Datasets subsection)
//   3 degree d(v) of the simple graph, then the order <+ (Preliminaries):
//     sort of (d(v), hash(v)) gives every vertex its rank
//   4 orient each edge from the lower to the higher rank and sort by
//     (source rank, target rank): rows ascend in the order <+
//   5 CSR with the time of each edge and the label of its target stored
//     beside it (Adj+^m of the Graph Storage subsection)
//   6 in-edge index: for every target q the list of (p, slot of q in p's row)
//     whose remaining row is non-empty -- the work the survey streams
//   7 plan: split each target's list into tiles and class targets by d+(q)
#include <algorithm>
#include <memory>
#include <vector>

#include "graph.hpp"
#include "plan.hpp"

using namespace tp;

namespace {

constexpr int kB = 256;

__device__ __forceinline__ uint64_t pair_key(uint32_t lo, uint32_t hi, int nb)
{
    return ((uint64_t)lo << nb) | hi;
}

// ------------------------------------------------------------ phase 0

// Graphs of a batch: graph g owns edges [eoff[g], eoff[g+1]) with local
// vertex ids < vcnt[g], which map to global ids voff[g] + local.
struct BatchMap {
    uint32_t n_graphs;
    const uint64_t *eoff;  // [n_graphs + 1]
    const uint32_t *voff;  // [n_graphs + 1]
};

// Pair keys through the two pair sorts: (g << 2 lb) | (a << lb) | b for two
// ids (vertices, then ranks) a, b local to graph g.  A batch's ranks are
// graph-major like its ids (graph g holds ranks voff[g] .. voff[g+1] - 1),
// so local ids and local ranks share the layout.  With local ids a batch's
// keys take 2 lb + gb bits (lb: bits of the largest graph's ids, gb: bits of
// the graph index) instead of 2 nb (nb: bits of all ids together): 47
// against 56 bits for the 20,000-graph batch, one radix pass fewer in each
// sort.  voff null: global ids, g = 0, lb = nb (single graphs, and batches
// whose local layout would be longer).
struct PairCode {
    int lb;
    const uint32_t *voff;
    __device__ __forceinline__ uint64_t pack(uint32_t g, uint32_t a, uint32_t b) const
    {
        return ((uint64_t)g << (2 * lb)) | ((uint64_t)a << lb) | b;
    }
    // first global id (or rank) of the key's graph
    __device__ __forceinline__ uint32_t base(uint64_t k) const { return voff ? voff[k >> (2 * lb)] : 0u; }
    __device__ __forceinline__ uint32_t hi(uint64_t k) const { return base(k) + (uint32_t)((k >> lb) & ((1ull << lb) - 1)); }
    __device__ __forceinline__ uint32_t lo(uint64_t k) const { return base(k) + (uint32_t)(k & ((1ull << lb) - 1)); }
};

__device__ __forceinline__ uint32_t graph_of_edge(const BatchMap &bm, size_t i)
{
    uint32_t a = 0, b = bm.n_graphs;  // eoff[a] <= i < eoff[b]
    while (b - a > 1) {
        const uint32_t mid = (a + b) >> 1;
        if (bm.eoff[mid] <= i) a = mid;
        else b = mid;
    }
    return a;
}

// Each workgroup canonicalises one contiguous span of `per_block` raw edges,
// so in a batch a thread finds the graph of its first edge by binary search
// and then only steps forward through the edge offsets.
// dbit = 1 (directed inputs) appends the direction of the raw edge to its
// key: 0 for lower id -> higher id, 1 for the reverse.
__global__ void k_canon(const uint32_t *src, const uint32_t *dst, const uint32_t *ts, size_t M, uint32_t n,
                        PairCode pc, int dbit, uint64_t sentinel, uint64_t *keys, uint32_t *vals,
                        unsigned long long *bad, unsigned long long *loops, BatchMap bm, size_t per_block)
{
    unsigned long long nbad = 0, nloop = 0;
    const size_t begin = blockIdx.x * per_block;
    const size_t end = begin + per_block < M ? begin + per_block : M;
    size_t i = begin + threadIdx.x;
    uint32_t g = 0;
    if (bm.n_graphs && i < end) g = graph_of_edge(bm, i);
    for (; i < end; i += blockDim.x) {
        uint32_t a = src[i], b = dst[i];
        bool ok;
        uint32_t kg = 0;  // graph index of the key (local layout)
        if (bm.n_graphs) {
            // local ids of graph g: kept local with the graph in the key, or
            // made global
            while (bm.eoff[g + 1] <= i) ++g;
            const uint32_t base = bm.voff[g], cnt = bm.voff[g + 1] - base;
            ok = a < cnt && b < cnt;
            if (pc.voff) {
                kg = g;
            } else {
                a += base;
                b += base;
            }
        } else {
            ok = a < n && b < n;
        }
        nbad += ok ? 0 : 1;
        uint64_t k;
        if (!ok || a == b) {
            k = sentinel;
            nloop += (ok && a == b) ? 1 : 0;
        } else {
            k = a < b ? pc.pack(kg, a, b) : pc.pack(kg, b, a);
            k = (k << dbit) | (uint64_t)(dbit && a > b);
        }
        keys[i] = k;
        vals[i] = ts ? ts[i] : 0u;
    }
    nbad = wave_sum(nbad);
    nloop = wave_sum(nloop);
    if (lane_id() == 0) {
        if (nbad) atomicAdd(bad, nbad);
        if (nloop) atomicAdd(loops, nloop);
    }
}

// ------------------------------------------------------------ phase 2

// A block takes a tile of kCompTile consecutive sorted pairs and wave w the
// tile's w-th part, 64 consecutive pairs at a time (lane l takes pair
// 64 j + l), so that every load is coalesced; the unique pairs leave in the
// same order.
constexpr int kCompItems = 16;
constexpr size_t kCompTile = (size_t)kB * kCompItems;
constexpr size_t kCompWave = (size_t)kWave * kCompItems;

// Is pair i the first of its run?  `k` is keys[i]; the previous key comes
// from the lane below, or from memory for lane 0.
// Keys carry dbit direction bits below the pair, which runs ignore.
__device__ __forceinline__ bool run_head(const uint64_t *keys, size_t i, size_t n, uint64_t k, int dbit)
{
    uint64_t prev = __shfl_up(k, 1, kWave);
    if (lane_id() == 0 && i < n) prev = i ? keys[i - 1] : ~k;
    return i < n && (prev >> dbit) != (k >> dbit);
}

// Unique pairs of this wave's part of the tile.
__device__ __forceinline__ uint64_t wave_heads(const uint64_t *keys, size_t n, size_t wbase, int dbit)
{
    uint64_t c = 0;
    for (int j = 0; j < kCompItems; ++j) {
        const size_t i = wbase + (size_t)j * kWave + lane_id();
        const uint64_t k = i < n ? keys[i] : 0ull;
        c += (uint64_t)__popcll(__ballot(run_head(keys, i, n, k, dbit)));
    }
    return c;
}

__global__ __launch_bounds__(kB) void k_dedup_count(const uint64_t *keys, size_t n, int dbit, uint64_t *tile_cnt)
{
    __shared__ uint64_t tmp[kB / kWave];
    const int w = threadIdx.x / kWave;
    const uint64_t c = wave_heads(keys, n, blockIdx.x * kCompTile + (size_t)w * kCompWave, dbit);
    if (lane_id() == 0) tmp[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int x = 0; x < kB / kWave; ++x) t += tmp[x];
        tile_cnt[blockIdx.x] = t;
    }
}

// Lane l's 64-bit value, in a scalar register (the builtin returns a signed
// 32-bit int: each half is widened as unsigned).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    return ((uint64_t)hi << 32) | lo;
}

// One pair per run with its earliest time; with direction bits (dbit = 1)
// also the directions of its copies (bit 0: lower -> higher id, bit 1: the
// reverse) into udir.  The wave keeps its 16 rounds of keys in registers
// from the count of its heads: the neighbours a head compares with come
// from the lanes beside it (or the next round's first lane), and only a run
// of copies is walked in memory.
__global__ __launch_bounds__(kB) void k_dedup_write(const uint64_t *keys, const uint32_t *vals, size_t n, int dbit,
                                                    const uint64_t *tile_off, uint64_t *ukey, uint32_t *uts,
                                                    uint8_t *udir)
{
    __shared__ uint64_t tmp[kB / kWave];
    const int w = threadIdx.x / kWave;
    const unsigned lane = lane_id();
    const size_t wbase = blockIdx.x * kCompTile + (size_t)w * kCompWave;
    uint64_t kk[kCompItems];
    uint64_t hm[kCompItems];  // each round's heads
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < kCompItems; ++j) {
        const size_t i = wbase + (size_t)j * kWave + lane;
        kk[j] = i < n ? keys[i] : 0ull;
        uint64_t prev = __shfl_up(kk[j], 1, kWave);
        if (j > 0) {
            const uint64_t last = readlane64(kk[j - 1], kWave - 1);
            if (lane == 0) prev = last;
        } else if (lane == 0 && i < n) {
            prev = i ? keys[i - 1] : ~kk[j];
        }
        hm[j] = __ballot(i < n && (prev >> dbit) != (kk[j] >> dbit));
        c += (uint64_t)__popcll(hm[j]);
    }
    if (lane == 0) tmp[w] = c;
    __syncthreads();
    uint64_t pos = tile_off[blockIdx.x];
    for (int x = 0; x < w; ++x) pos += tmp[x];
#pragma unroll
    for (int j = 0; j < kCompItems; ++j) {
        const size_t i = wbase + (size_t)j * kWave + lane;
        const uint64_t k = kk[j];
        // the key after this one: the next lane's, the next round's first, or memory
        uint64_t next = __shfl_down(k, 1, kWave);
        if (j + 1 < kCompItems) {
            const uint64_t first = readlane64(kk[j + 1], 0);
            if (lane == kWave - 1) next = first;
        } else if (lane == kWave - 1) {
            next = i + 1 < n ? keys[i + 1] : 0ull;
        }
        const uint64_t b = hm[j];
        if ((b >> lane) & 1ull) {
            // the earliest time of the run, and its directions
            const uint64_t pk = k >> dbit;
            uint32_t t = vals[i];
            uint32_t d = 1u << (k & (uint64_t)dbit);
            if (i + 1 < n && (next >> dbit) == pk) {
                for (size_t x = i + 1; x < n && (keys[x] >> dbit) == pk; ++x) {
                    t = min(t, vals[x]);
                    d |= 1u << (keys[x] & (uint64_t)dbit);
                }
            }
            const uint64_t at = pos + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
            ukey[at] = pk;
            uts[at] = t;
            if (udir) udir[at] = (uint8_t)d;
        }
        pos += (uint64_t)__popcll(b);
    }
}

// ------------------------------------------------------------ phase 3

// Add the lengths of the runs of equal values among a wave's 64 values
// (sorted; lanes with ok == false form a suffix) to cnt[value]: one atomic
// per run, to increasing addresses.
__device__ __forceinline__ void add_runs(uint64_t v, bool ok, uint32_t *cnt)
{
    const unsigned lane = lane_id();
    const uint64_t prev = __shfl_up(v, 1, kWave);
    const bool head = ok && (lane == 0 || prev != v);
    const uint64_t heads = __ballot(head);
    const uint32_t valid = (uint32_t)__popcll(__ballot(ok));
    if (head) {
        const uint64_t above = lane == 63 ? 0ull : (heads & (~0ull << (lane + 1)));
        const uint32_t next = above ? (uint32_t)__ffsll((long long)above) - 1 : valid;
        atomicAdd(&cnt[v], next - lane);
    }
}

// d(v) counts each unique pair at both ends.  The pairs are sorted by their
// lower end, so that half is counted by runs; the higher ends are written
// out here (one read of the pairs for both), sorted on their own (a 32-bit
// radix sort) and counted the same way by k_degree_runs, instead of one
// scattered atomic per pair.
__global__ void k_degree_low(const uint64_t *ukey, size_t m, PairCode pc, uint32_t *deg, uint32_t *hi)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < m; base += stride) {
        const size_t i = base + lane_id();
        const bool ok = i < m;
        const uint64_t k = ok ? ukey[i] : 0ull;
        add_runs(ok ? pc.hi(k) : ~0ull, ok, deg);
        if (ok) hi[i] = pc.lo(k);
    }
}

__global__ void k_degree_runs(const uint32_t *v, size_t m, uint32_t *deg)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < m; base += stride) {
        const size_t i = base + lane_id();
        const bool ok = i < m;
        add_runs(ok ? v[i] : ~0ull, ok, deg);
    }
}

template <class T>
__global__ void k_max(const T *x, size_t n, unsigned long long *out)
{
    unsigned long long mx = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        mx = max(mx, (unsigned long long)x[i]);
    mx = wave_max(mx);
    if (lane_id() == 0 && mx) atomicMax(out, mx);
}

// A bijection of [0, 2^nb): xor-shifts and odd multiplications modulo 2^nb.
__device__ __forceinline__ uint32_t tie_mix(uint32_t x, int nb)
{
    const uint64_t mask = (nb >= 32) ? 0xffffffffull : ((1ull << nb) - 1);
    const int s = (nb + 1) / 2;
    uint64_t y = x;
    y ^= y >> s;
    y = (y * 0x9e3779b1ull) & mask;
    y ^= y >> s;
    y = (y * 0x85ebca6bull) & mask;
    y ^= y >> s;
    return (uint32_t)y;
}

// graph of vertex v in a batch: voff[g] <= v < voff[g + 1]
__device__ __forceinline__ uint32_t graph_of_vertex(const uint32_t *voff, uint32_t n_graphs, uint32_t v)
{
    uint32_t a = 0, b = n_graphs;
    while (b - a > 1) {
        const uint32_t mid = (a + b) >> 1;
        if (voff[mid] <= v) a = mid;
        else b = mid;
    }
    return a;
}

// Sort key of the degree order: (d(v), hash(v)).  In a batch the graph id
// sits above them, so that every graph owns a contiguous range of ranks (the
// graphs share no edge, so the order between graphs is free).
__global__ void k_rank_keys(const uint32_t *deg, uint32_t n, int nb, int gshift, const uint32_t *voff,
                            uint32_t n_graphs, uint32_t tie, uint64_t *rkey, uint32_t *rval)
{
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const uint32_t h = tie == TP_TIE_ID ? (uint32_t)v : tie_mix((uint32_t)v, nb);
        uint64_t key = ((uint64_t)deg[v] << nb) | h;
        if (voff) key |= (uint64_t)graph_of_vertex(voff, n_graphs, (uint32_t)v) << gshift;
        rkey[v] = key;
        rval[v] = (uint32_t)v;
    }
}

__global__ void k_rank_scatter(const uint32_t *perm, uint32_t n, const uint8_t *vlab, uint32_t *rank, uint8_t *rlab)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t v = perm[i];
        rank[v] = (uint32_t)i;
        rlab[i] = vlab ? vlab[v] : 0;
    }
}

// ceil(log2 d) for d >= 2 (the bit length of d - 1); 0 for d <= 1; cap 31
__device__ __forceinline__ uint32_t degree_bin(uint32_t d)
{
    if (d <= 1) return 0;
    const uint32_t b = 32u - (uint32_t)__clz(d - 1);
    return b > 31 ? 31 : b;
}

// Ranks are in degree order, so the degree bins are ranges of ranks:
// first[k] = the first rank whose bin is >= k (first[] is pre-filled with
// 2^32 - 1 for bins above the largest).  Rank i writes the bins it opens.
// In a batch each graph's ranks are a range of their own in degree order,
// so each graph g gets its own 32 bounds at first[32 g + k], and a graph's
// first rank opens every bin up to its own.  Rank i's degree (bits
// [nb, gshift)) and graph (bits from gshift) are read from its sorted order
// key, in rank order.
__global__ void k_dbin_rank(const uint64_t *skey, uint32_t n, int nb, int gshift, bool batch, uint32_t *first)
{
    const uint64_t dmask = (1ull << (gshift - nb)) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t key = skey[i];
        const uint32_t b = degree_bin((uint32_t)((key >> nb) & dmask));
        const uint32_t g = batch ? (uint32_t)(key >> gshift) : 0u;
        uint64_t pkey = 0;
        if (i) pkey = skey[i - 1];
        const bool opens = i == 0 || (batch && (uint32_t)(pkey >> gshift) != g);
        const int prev = opens ? -1 : (int)degree_bin((uint32_t)((pkey >> nb) & dmask));
        for (int k = prev + 1; k <= (int)b; ++k) first[(size_t)g * 32 + k] = (uint32_t)i;
    }
}

// The same boundaries as CSR slots: rows are laid out by rank.
__global__ void k_dbin_slot(const uint32_t *first, const uint64_t *rowptr, size_t count, uint64_t *slot)
{
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
        slot[k] = first[k] == 0xffffffffu ? ~0ull : rowptr[first[k]];
}

__global__ void fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// graph id of every rank in a batch: the bits above gshift of its sorted
// order key
__global__ void k_rank_graph(const uint64_t *skey, uint32_t n, int gshift, uint32_t *rank_gid)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        rank_gid[i] = (uint32_t)(skey[i] >> gshift);
}

// ------------------------------------------------------------ phase 4

// With directions (udir set), the oriented key carries two bits below the
// pair: bit 0 for the arc source -> target of the oriented edge, bit 1 for
// the reverse.
// (The times stay where the dedup wrote them: the orientation sort takes
// them as its values in place, so that they are not copied here.)
__global__ void k_orient(const uint64_t *ukey, const uint8_t *udir, size_t m, PairCode pc, const uint32_t *rank,
                         uint64_t *okey)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = ukey[i];
        const uint32_t base = pc.base(k);
        const uint32_t a = rank[pc.hi(k)], b = rank[pc.lo(k)];
        const uint32_t s = min(a, b), t = max(a, b);
        // local ranks of the key's graph (its ranks start at its first id)
        uint64_t o = pc.pack((uint32_t)(pc.voff ? k >> (2 * pc.lb) : 0u), s - base, t - base);
        if (udir) {
            // udir is relative to lower id -> higher id; a is the lower id's rank
            const uint32_t d = udir[i];
            o = (o << 2) | (a < b ? d : (((d & 1u) << 1) | (d >> 1)));
        }
        okey[i] = o;
    }
}



// ------------------------------------------------------------ phase 5

// The oriented pairs sorted by source: position i is CSR slot i.  One read
// of them writes each slot's target, its label, its source and (directed
// builds) the two direction bits below the pair into edir, and counts d+(s):
// each wave adds one count per run of equal sources among its 64 pairs, to
// increasing addresses.
__global__ void k_csr(const uint64_t *okey, size_t m, PairCode pc, const uint8_t *rlab, uint32_t *col, uint8_t *tlab,
                      uint32_t *srow, uint8_t *edir, uint32_t *dplus)
{
    const int dshift = edir ? 2 : 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < m; base += stride) {
        const size_t i = base + lane_id();
        const bool ok = i < m;
        const uint64_t k = ok ? okey[i] : 0ull;
        const uint32_t src = pc.hi(k >> dshift);
        add_runs(ok ? (uint64_t)src : ~0ull, ok, dplus);
        if (ok) {
            const uint32_t t = pc.lo(k >> dshift);
            col[i] = t;
            tlab[i] = rlab[t];
            srow[i] = src;
            if (edir) edir[i] = (uint8_t)(k & 3u);
        }
    }
}

__global__ void k_row_stats(const uint64_t *rowptr, uint32_t n, unsigned long long *wedges,
                            unsigned long long *dplus_max)
{
    unsigned long long w = 0, mx = 0;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        const uint64_t d = rowptr[v + 1] - rowptr[v];
        w += d ? d * (d - 1) / 2 : 0;
        mx = max(mx, (unsigned long long)d);
    }
    w = wave_sum(w);
    mx = wave_max(mx);
    if (lane_id() == 0) {
        if (w) atomicAdd(wedges, w);
        if (mx) atomicMax(dplus_max, mx);
    }
}

// ------------------------------------------------------------ phase 6

// The wedges (p, q, r) of the oriented edge p -> q at slot k are the slots
// after k in p's row; they can close only if q has out-neighbours.
__device__ __forceinline__ uint32_t rest_len(const uint64_t *rowptr, uint32_t s, size_t k)
{
    return (uint32_t)(rowptr[s + 1] - k - 1);
}

// One bit per vertex: whether its row is non-empty (bit v & 63 of word
// v >> 6).  At one bit per vertex the array stays in cache, where the row
// pointers of random targets would not.
__global__ void k_has_out(const uint64_t *rowptr, uint32_t n, uint64_t *bits)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < n; base += stride) {
        const size_t v = base + lane_id();
        const bool b = v < n && rowptr[v + 1] > rowptr[v];
        const uint64_t word = __ballot(b);
        if (lane_id() == 0) bits[base >> 6] = word;
    }
}

// Key of each oriented edge for the in-edge sort: (q << kbits) | k, with q
// replaced by n (sorted past every target) when the edge has no wedge to
// check; and the record payload that travels with it through the sort: the
// length of the rest of p's row after slot k (< 2^22) | label(p) << 24.
// Counts the edges kept.  Slots are in row order, so every read here walks
// memory forwards, but for the bit of q.
__global__ void k_in_keys(const uint32_t *srow, const uint32_t *col, const uint64_t *rowptr, const uint64_t *has_out,
                          const uint8_t *rlab, size_t m, int kbits, uint32_t n, uint64_t *key, uint32_t *pay,
                          unsigned long long *kept)
{
    unsigned long long c = 0;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < m; k += (size_t)gridDim.x * blockDim.x) {
        const uint32_t s = srow[k], t = col[k];
        const uint32_t rest = rest_len(rowptr, s, k);
        const bool ok = rest > 0 && ((has_out[t >> 6] >> (t & 63)) & 1ull);
        key[k] = ((uint64_t)(ok ? t : n) << kbits) | k;
        pay[k] = rest | ((uint32_t)rlab[s] << 24);
        c += ok ? 1 : 0;
    }
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(kept, c);
}

// In-edges and wedge checks of every target (the sum of the remaining row
// lengths of its in-edges).  In-edges of one target are consecutive, so each
// wave adds one partial sum per run of equal targets.
__global__ void k_in_work(const uint64_t *key, const uint32_t *pay, uint64_t n_in, int kbits,
                          unsigned long long *work, uint32_t *count)
{
    const unsigned lane = lane_id();
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = blockIdx.x * (size_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < n_in; base += stride) {
        const size_t i = base + lane;
        const bool ok = i < n_in;
        uint64_t t = ~0ull, len = 0;
        if (ok) {
            t = key[i] >> kbits;
            len = pay[i] & 0xffffffu;
        }
        const uint64_t tprev = __shfl_up(t, 1, kWave);
        const bool head = ok && (lane == 0 || tprev != t);
        const uint64_t heads = __ballot(head);
        const uint64_t incl = wave_incl_scan(len);
        // the lane where this lane's run starts, and the prefix before it
        const uint64_t upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
        const int start = 63 - __clzll(upto);
        const uint64_t before = __shfl(incl - len, start, kWave);
        const uint64_t tnext = __shfl_down(t, 1, kWave);
        const bool last = ok && (lane == 63 || i + 1 >= n_in || tnext != t);
        if (last) {
            atomicAdd(&work[t], (unsigned long long)(incl - before));
            atomicAdd(&count[t], lane - (unsigned)start + 1u);
        }
    }
}

// ------------------------------------------------------------ phase 7

__device__ __forceinline__ int class_of(uint64_t dq)
{
    return dq <= kTinyMaxDeg ? kClassTiny
                             : (dq <= kSmallMaxDeg ? kClassSmall : (dq <= kLargeMaxDeg ? kClassLarge : kClassHuge));
}

// Tile caps of each class: records per tile and wedge checks per tile.
struct TileCaps {
    uint32_t rec[kNumClasses];
    uint64_t work[kNumClasses];
};

__device__ __forceinline__ uint32_t tiles_of(uint64_t cnt, uint64_t work, uint32_t rec_cap, uint64_t work_cap)
{
    if (cnt == 0) return 0;
    const uint64_t a = (cnt + rec_cap - 1) / rec_cap;
    const uint64_t b = (work + work_cap - 1) / work_cap;
    uint64_t t = a > b ? a : b;
    if (t > cnt) t = cnt;
    return (uint32_t)t;
}

// Records of piece j of target q (pieces of huge targets; pos[] is the
// exclusive scan of the cut flags, fbase[] the first flag of each target):
// [first, first + count) in the piece record arrays.
__device__ __forceinline__ void piece_records(const uint64_t *fbase, const uint64_t *pos, size_t q, uint32_t j,
                                              uint64_t cnt, uint64_t &first, uint64_t &count)
{
    first = pos[fbase[q] + j * cnt];
    count = pos[fbase[q] + (j + 1) * cnt] - first;
}

__global__ void k_plan_count(const uint64_t *cptr, const unsigned long long *work, const uint64_t *rowptr,
                             const uint64_t *fbase, const uint64_t *pos, uint32_t n, TileCaps caps,
                             uint32_t *tcnt /* [classes][n] */)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const uint64_t cnt = cptr[q + 1] - cptr[q];
        const int c = class_of(rowptr[q + 1] - rowptr[q]);
        uint32_t rc = caps.rec[0];
        uint64_t wc = caps.work[0];
#pragma unroll
        for (int i = 1; i < kNumClasses; ++i) {
            if (i == c) {
                rc = caps.rec[i];
                wc = caps.work[i];
            }
        }
        uint32_t t = 0;
        if (c == kClassHuge && cnt) {
            // each piece of Adj+(q) has its own records and tiles; it sees
            // about 1/S of the target's wedge checks
            const uint32_t S = piece_count(rowptr[q + 1] - rowptr[q]);
            for (uint32_t j = 0; j < S; ++j) {
                uint64_t first, count;
                piece_records(fbase, pos, q, j, cnt, first, count);
                t += tiles_of(count, (work[q] + S - 1) / S, rc, wc);
            }
        } else {
            t = tiles_of(cnt, work[q], rc, wc);
        }
        for (int i = 0; i < kNumClasses; ++i) tcnt[(size_t)i * n + q] = (i == c) ? t : 0u;
    }
}

// The tiles of target q, dealing its records round-robin; for a huge
// target, the tiles of each piece in turn over that piece's records.
__global__ void k_plan_write(const uint64_t *cptr, const unsigned long long *work, const uint64_t *rowptr,
                             const uint64_t *fbase, const uint64_t *pos, const uint64_t *tile_off,
                             const uint32_t *tcnt, uint32_t n, TileCaps caps, int cls, TileDesc *tiles)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const uint32_t t = tcnt[q];
        if (!t) continue;
        const uint64_t cnt = cptr[q + 1] - cptr[q];
        uint64_t at = tile_off[q];
        auto deal = [&](uint64_t first, uint64_t count, uint32_t tj, uint32_t piece) {
            for (uint32_t i = 0; i < tj; ++i) {
                TileDesc d;
                d.q = (uint32_t)q;
                d.cnt = (uint32_t)((count - i + tj - 1) / tj);  // records i, i + tj, ...
                d.e0 = first + i;
                d.stride = tj;
                d.piece = piece;
                tiles[at++] = d;
            }
        };
        if (cls == kClassHuge) {
            const uint32_t S = piece_count(rowptr[q + 1] - rowptr[q]);
            for (uint32_t j = 0; j < S; ++j) {
                uint64_t first, count;
                piece_records(fbase, pos, q, j, cnt, first, count);
                deal(first, count, tiles_of(count, (work[q] + S - 1) / S, caps.rec[cls], caps.work[cls]), j);
            }
        } else {
            deal(cptr[q], cnt, t, 0);
        }
    }
}

// ---- records of huge targets, cut to the pieces of Adj+(q)

// Number of the `len` sorted ranks at `a` that are below x (binary search).
__device__ __forceinline__ uint32_t count_below(const uint32_t *a, uint32_t len, uint32_t x)
{
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Cut flags per target: S * (records) for a huge target with records, else
// none; the huge targets with records are listed (in no particular order;
// at most m / (kLargeMaxDeg + 1) targets have d+ above kLargeMaxDeg).
__global__ void k_piece_slots(const uint64_t *cptr, const uint64_t *rowptr, uint32_t n, uint32_t *slots,
                              uint32_t *list, unsigned long long *n_list)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const uint64_t dq = rowptr[q + 1] - rowptr[q], cnt = cptr[q + 1] - cptr[q];
        const bool huge = class_of(dq) == kClassHuge && cnt > 0;
        slots[q] = huge ? (uint32_t)(piece_count(dq) * cnt) : 0u;
        if (huge) list[atomicAdd(n_list, 1ull)] = (uint32_t)q;
    }
}

// For every record p -> q of a listed huge target (grid row y: targets y,
// y + gridDim.y, ...) and every piece j of Adj+(q): the candidates of the
// record (the rest of p's row, sorted by rank) whose ranks lie in the
// piece's range [first key of piece j, first key of piece j + 1).
// WRITE false: at f = fbase[q] + j cnt + r (r the record's place among q's
// records) flag[f] = (any candidates) and cut[f] = the end of the piece's
// candidates in the record.  WRITE true: the record cut to the piece, from
// cut[], at pos[f].
template <bool WRITE>
__global__ void k_piece_cut(const uint64_t *inkey, const uint32_t *inpay, int kbits, const uint32_t *list,
                            uint64_t n_list, const uint64_t *cptr, const uint64_t *rowptr, const uint32_t *col,
                            const uint64_t *fbase, uint32_t *flag, uint32_t *cut, const uint64_t *pos,
                            uint64_t *pkey, uint32_t *ppay)
{
    const uint64_t kmask = (1ull << kbits) - 1;
    for (uint64_t t = blockIdx.y; t < n_list; t += gridDim.y) {
        const uint64_t q = list[t];
        const uint64_t kq = rowptr[q], dq = rowptr[q + 1] - kq;
        const uint32_t S = piece_count(dq), psz = piece_size(dq);
        const uint64_t c0 = cptr[q], cnt = cptr[q + 1] - c0;
        for (uint64_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < cnt; r += (size_t)gridDim.x * blockDim.x) {
            const uint64_t key = inkey[c0 + r];
            const uint64_t k = key & kmask;
            const uint32_t pay = inpay[c0 + r], len = pay & 0xffffffu;
            const uint32_t *cand = col + k + 1;
            uint32_t lo = 0;
            for (uint32_t j = 0; j < S; ++j) {
                const uint64_t f = fbase[q] + j * cnt + r;
                uint32_t hi;
                if (!WRITE) {
                    hi = j + 1 < S ? count_below(cand, len, col[kq + (uint64_t)(j + 1) * psz]) : len;
                    flag[f] = hi > lo ? 1u : 0u;
                    cut[f] = hi;
                } else if ((hi = cut[f]) > lo) {
                    // q + lo < 2n fits above bit kbits, as q <= n does
                    pkey[pos[f]] = ((q + lo) << kbits) | k;
                    ppay[pos[f]] = (pay & 0xff000000u) | (hi - lo);
                }
                lo = hi;
            }
        }
    }
}

// Per-class totals of the plan: records, staged out-list entries, probes;
// then the probes of all targets and the number of targets with any.
__global__ void k_plan_stats(const uint64_t *cptr, const unsigned long long *work, const uint64_t *rowptr,
                             const uint64_t *fbase, const uint64_t *pos, const uint32_t *tcnt, uint32_t n,
                             TileCaps caps, unsigned long long *out /* [3][classes], probes, targets */)
{
    unsigned long long rec[kNumClasses] = {}, stg[kNumClasses] = {}, prb[kNumClasses] = {}, wall = 0, wnz = 0;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const unsigned long long wq = work[q];
        wall += wq;
        wnz += wq ? 1 : 0;
        const uint64_t dq = rowptr[q + 1] - rowptr[q];
        const int c = class_of(dq);
        const uint32_t t = tcnt[(size_t)c * n + q];
        if (!t) continue;
        // a huge target: the records cut to its pieces, each piece staged by
        // each of its tiles
        uint64_t nrec = cptr[q + 1] - cptr[q], staged = (uint64_t)t * dq;
        if (c == kClassHuge) {
            const uint32_t S = piece_count(dq), psz = piece_size(dq);
            const uint64_t cnt = nrec;
            nrec = 0;
            staged = 0;
            for (uint32_t j = 0; j < S; ++j) {
                uint64_t first, count;
                piece_records(fbase, pos, q, j, cnt, first, count);
                nrec += count;
                staged += (uint64_t)tiles_of(count, (work[q] + S - 1) / S, caps.rec[c], caps.work[c]) *
                          min((uint64_t)psz, dq - (uint64_t)j * psz);
            }
        }
#pragma unroll
        for (int i = 0; i < kNumClasses; ++i) {
            if (i == c) {
                rec[i] += nrec;
                stg[i] += staged;
                prb[i] += wq;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kNumClasses; ++i) {
        const unsigned long long a = wave_sum(rec[i]), b = wave_sum(stg[i]), c = wave_sum(prb[i]);
        if (lane_id() == 0) {
            if (a) atomicAdd(&out[0 * kNumClasses + i], a);
            if (b) atomicAdd(&out[1 * kNumClasses + i], b);
            if (c) atomicAdd(&out[2 * kNumClasses + i], c);
        }
    }
    wall = wave_sum(wall);
    wnz = wave_sum(wnz);
    if (lane_id() == 0) {
        if (wall) atomicAdd(&out[3 * kNumClasses], wall);
        if (wnz) atomicAdd(&out[3 * kNumClasses + 1], wnz);
    }
}

template <class T>
T read_scalar(const T *dev, hipStream_t s)
{
    T v;
    TP_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    return v;
}

template <class T>
const T *to_device(const T *p, size_t n, uint32_t space, DArray<T> &hold, hipStream_t s)
{
    if (!p || space == TP_MEM_DEVICE) return p;
    hold.reset(n, s);
    if (n) TP_HIP(hipMemcpyAsync(hold.get(), p, n * sizeof(T), hipMemcpyHostToDevice, s));
    return hold.get();
}

}  // namespace

// ================================================================ plan

uint64_t graph_bytes(const tp_graph *g)
{
    uint64_t b = g->rowptr.bytes() + g->col.bytes() + g->ets.bytes() + g->tlab.bytes() + g->rlab.bytes() +
                 g->perm.bytes() + g->inkey.bytes() + g->inpay.bytes() + g->rank_gid.bytes() +
                 g->dbin_rank.bytes() + g->dbin_slot.bytes() + g->edir.bytes() + g->piece_key.bytes() +
                 g->piece_pay.bytes();
    for (int c = 0; c < kNumClasses; ++c) b += g->tiles[c].bytes();
    return b;
}

// Cut the tiles of every class with the caps of `cfg` and record the plan's
// statistics.  The work of each target (in-edges and wedge checks) is
// recomputed from the in-edge index.
void plan_graph(tp_graph *g, const PlanCfg &cfg, hipStream_t s)
{
    const uint32_t n = g->n;
    DArray<unsigned long long> work(n, s);
    DArray<uint64_t> cptr((size_t)n + 1, s);
    {
        DArray<uint32_t> incnt(n, s);
        TP_HIP(hipMemsetAsync(incnt.get(), 0, n * sizeof(uint32_t), s));
        TP_HIP(hipMemsetAsync(work.get(), 0, n * sizeof(unsigned long long), s));
        if (g->n_in) {
            k_in_work<<<grid_for(g->n_in, kB), kB, 0, s>>>(g->inkey.get(), g->inpay.get(), g->n_in, (int)g->kbits,
                                                           work.get(), incnt.get());
            TP_CHECK_LAUNCH();
        }
        scan_u32_to_u64(incnt.get(), cptr.get(), n, s);
    }
    // the records of huge targets cut to the pieces of Adj+(q): a flag per
    // (record, piece), laid out target by target and piece by piece; the
    // scan of the flags places every cut record
    DArray<uint64_t> fbase, pos;
    g->piece_key.release();
    g->piece_pay.release();
    g->n_piece_recs = 0;
    if (g->n_in && g->stats.dplus_max > kLargeMaxDeg) {
        fbase.reset((size_t)n + 1, s);
        DArray<uint32_t> list(g->m / (kLargeMaxDeg + 1) + 1, s);
        DArray<unsigned long long> n_list(1, s);
        TP_HIP(hipMemsetAsync(n_list.get(), 0, sizeof(unsigned long long), s));
        {
            DArray<uint32_t> slots(n, s);
            k_piece_slots<<<grid_for(n, kB), kB, 0, s>>>(cptr.get(), g->rowptr.get(), n, slots.get(), list.get(),
                                                         n_list.get());
            TP_CHECK_LAUNCH();
            scan_u32_to_u64(slots.get(), fbase.get(), n, s);
        }
        const uint64_t nf = read_scalar(fbase.get() + n, s);
        const uint64_t nh = read_scalar(n_list.get(), s);
        // a grid row per listed target (strided), its records across the row
        const dim3 grid(64, (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(nh, 4096)));
        pos.reset(nf + 1, s);
        DArray<uint32_t> cut(std::max<uint64_t>(nf, 1), s);
        {
            DArray<uint32_t> flag(std::max<uint64_t>(nf, 1), s);
            if (nh) {
                k_piece_cut<false><<<grid, kB, 0, s>>>(g->inkey.get(), g->inpay.get(), (int)g->kbits, list.get(), nh,
                                                       cptr.get(), g->rowptr.get(), g->col.get(), fbase.get(),
                                                       flag.get(), cut.get(), nullptr, nullptr, nullptr);
                TP_CHECK_LAUNCH();
            }
            scan_u32_to_u64(flag.get(), pos.get(), nf, s);
        }
        const uint64_t nr = read_scalar(pos.get() + nf, s);
        g->n_piece_recs = nr;
        g->piece_key.reset(std::max<uint64_t>(nr, 1), s);
        g->piece_pay.reset(std::max<uint64_t>(nr, 1), s);
        if (nr) {
            k_piece_cut<true><<<grid, kB, 0, s>>>(g->inkey.get(), g->inpay.get(), (int)g->kbits, list.get(), nh,
                                                  cptr.get(), g->rowptr.get(), g->col.get(), fbase.get(), nullptr,
                                                  cut.get(), pos.get(), g->piece_key.get(), g->piece_pay.get());
            TP_CHECK_LAUNCH();
        }
    }
    TileCaps caps;
    for (int c = 0; c < kNumClasses; ++c) {
        caps.rec[c] = cfg.tile_records[c];
        caps.work[c] = kTileWorkPerRecord * cfg.tile_records[c];
    }
    DArray<uint32_t> tcnt((size_t)kNumClasses * n, s);
    k_plan_count<<<grid_for(n, kB), kB, 0, s>>>(cptr.get(), work.get(), g->rowptr.get(), fbase.get(), pos.get(), n,
                                                caps, tcnt.get());
    TP_CHECK_LAUNCH();
    for (int c = 0; c < kNumClasses; ++c) {
        DArray<uint64_t> toff((size_t)n + 1, s);
        scan_u32_to_u64(tcnt.get() + (size_t)c * n, toff.get(), n, s);
        const uint64_t nt = read_scalar(toff.get() + n, s);
        g->n_tiles[c] = nt;
        g->tiles[c].reset(std::max<uint64_t>(nt, 1), s);
        if (nt) {
            k_plan_write<<<grid_for(n, kB), kB, 0, s>>>(cptr.get(), work.get(), g->rowptr.get(), fbase.get(),
                                                        pos.get(), toff.get(), tcnt.get() + (size_t)c * n, n, caps,
                                                        c, g->tiles[c].get());
            TP_CHECK_LAUNCH();
        }
    }
    // per class: records, staged entries, probes; then all probes and active targets
    constexpr int kStat = 3 * kNumClasses;
    DArray<unsigned long long> pst(kStat + 2, s);
    TP_HIP(hipMemsetAsync(pst.get(), 0, (kStat + 2) * sizeof(unsigned long long), s));
    k_plan_stats<<<grid_for(n, kB), kB, 0, s>>>(cptr.get(), work.get(), g->rowptr.get(), fbase.get(), pos.get(),
                                                tcnt.get(), n, caps, pst.get());
    TP_CHECK_LAUNCH();
    unsigned long long h[kStat + 2];
    TP_HIP(hipMemcpyAsync(h, pst.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    g->stats.n_tiles = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        g->stats.class_tiles[c] = g->n_tiles[c];
        g->stats.class_records[c] = h[c];
        g->stats.class_staged[c] = h[kNumClasses + c];
        g->stats.class_probes[c] = h[2 * kNumClasses + c];
        g->stats.n_tiles += g->n_tiles[c];
    }
    g->stats.probes = h[kStat];
    g->stats.n_targets = h[kStat + 1];
    g->plan = cfg;
}

// ================================================================ build

struct HostBatch {
    uint32_t n_graphs = 0;
    std::vector<uint64_t> eoff;  // [n_graphs + 1]
    std::vector<uint32_t> voff;  // [n_graphs + 1]
};

static void build_impl(const tp_edge_list *el, hipStream_t s, tp_graph **out, const HostBatch *hb = nullptr)
{
    if (!el || !out) fail(TP_ERR_INVALID, "tripoll_build: NULL argument");
    if (el->mem_space != TP_MEM_HOST && el->mem_space != TP_MEM_DEVICE)
        fail(TP_ERR_INVALID, "tripoll_build: mem_space must be TP_MEM_HOST or TP_MEM_DEVICE");
    if (el->tie_hash != TP_TIE_MIX && el->tie_hash != TP_TIE_ID)
        fail(TP_ERR_INVALID, "tripoll_build: unknown tie_hash");
    if (el->n_vertices == 0 || el->n_vertices >= 0xffffffffu)
        fail(TP_ERR_INVALID, "tripoll_build: n_vertices must be in [1, 2^32-1)");
    if (el->n_edges > 0 && (!el->src || !el->dst)) fail(TP_ERR_INVALID, "tripoll_build: NULL src/dst");
    if (el->flags & ~TP_EDGES_DIRECTED) fail(TP_ERR_INVALID, "tripoll_build: unknown flags");

    const uint32_t n = el->n_vertices;
    const size_t M = el->n_edges;
    const int nb = std::max(1, bits_for((uint64_t)n - 1));
    // directed inputs carry one direction bit per raw edge through the pair
    // sort and two per oriented edge through the orientation sort
    const bool directed = (el->flags & TP_EDGES_DIRECTED) != 0;
    const int dbit = directed ? 1 : 0, dbit2 = directed ? 2 : 0;
    if (2 * nb + dbit2 > 64) fail(TP_ERR_UNSUPPORTED, "tripoll_build: too many vertices for directed keys");
    // pair keys: a batch keeps its ids local (graph index on top) when that
    // layout is the shorter one
    int kb = 2 * nb;  // bits of a pair key
    int lb = nb;      // bits of one id in it
    bool local_keys = false;
    if (hb && hb->n_graphs > 1) {
        uint32_t vmax = 1;
        for (uint32_t i = 0; i < hb->n_graphs; ++i) vmax = std::max(vmax, hb->voff[i + 1] - hb->voff[i]);
        const int l = std::max(1, bits_for((uint64_t)vmax - 1));
        const int gb = bits_for((uint64_t)hb->n_graphs - 1);
        if (2 * l + gb < kb) {
            local_keys = true;
            lb = l;
            kb = 2 * l + gb;
        }
    }
    const uint64_t sentinel = (kb + dbit >= 64) ? ~0ull : ((1ull << (kb + dbit)) - 1);

    auto g = std::make_unique<tp_graph>();
    TP_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->nbits = (uint32_t)nb;

    hipEvent_t ev[9];
    for (auto &e : ev) TP_HIP(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { for (int i = 0; i < 9; ++i) (void)hipEventDestroy(e[i]); }
    } evg{ev};
    TP_HIP(hipEventRecord(ev[0], s));

    // ---- phase 0: upload and canonicalise
    DArray<uint32_t> h_src, h_dst, h_ts;
    DArray<uint8_t> h_lab;
    const uint32_t *src = to_device(el->src, M, el->mem_space, h_src, s);
    const uint32_t *dst = to_device(el->dst, M, el->mem_space, h_dst, s);
    const uint32_t *ts = to_device(el->edge_time, M, el->mem_space, h_ts, s);
    const uint8_t *vlab = to_device(el->vertex_label, n, el->mem_space, h_lab, s);

    // bad ids, self-loops, d_max, max label, wedges, d+_max, probes, active targets
    DArray<unsigned long long> counters(8, s);
    TP_HIP(hipMemsetAsync(counters.get(), 0, 8 * sizeof(unsigned long long), s));
    unsigned long long *c_bad = counters.get(), *c_loop = c_bad + 1, *c_dmax = c_bad + 2, *c_lab = c_bad + 3,
                       *c_wedge = c_bad + 4, *c_dpmax = c_bad + 5;

    const size_t Mcap = std::max<size_t>(M, 1);
    DArray<uint64_t> keyA(Mcap, s), keyB(Mcap, s);
    // (the value buffers end with room for the row pad: one of them becomes
    // the graph's edge times)
    DArray<uint32_t> valA(Mcap + kRowPad, s), valB(Mcap + kRowPad, s);
    BatchMap bm{0, nullptr, nullptr};
    DArray<uint64_t> d_eoff;
    DArray<uint32_t> d_voff;
    if (hb) {
        d_eoff.reset(hb->n_graphs + 1, s);
        d_voff.reset(hb->n_graphs + 1, s);
        TP_HIP(hipMemcpyAsync(d_eoff.get(), hb->eoff.data(), (hb->n_graphs + 1) * sizeof(uint64_t),
                              hipMemcpyHostToDevice, s));
        TP_HIP(hipMemcpyAsync(d_voff.get(), hb->voff.data(), (hb->n_graphs + 1) * sizeof(uint32_t),
                              hipMemcpyHostToDevice, s));
        bm = BatchMap{hb->n_graphs, d_eoff.get(), d_voff.get()};
    }
    const PairCode pc{lb, local_keys ? d_voff.get() : nullptr};
    if (M) {
        const unsigned blocks = grid_for(M, kB);
        const size_t per_block = (M + blocks - 1) / blocks;
        k_canon<<<blocks, kB, 0, s>>>(src, dst, ts, M, n, pc, dbit, sentinel, keyA.get(), valA.get(), c_bad, c_loop, bm,
                                      per_block);
        TP_CHECK_LAUNCH();
    }
    unsigned long long hc[2];
    TP_HIP(hipMemcpyAsync(hc, counters.get(), 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    TP_HIP(hipStreamSynchronize(s));
    if (hc[0]) fail(TP_ERR_INVALID, "tripoll_build: " + std::to_string(hc[0]) + " edge endpoints >= n_vertices");
    h_src.release();
    h_dst.release();
    h_ts.release();
    const size_t Mv = M - (size_t)hc[1];  // edges that are not self-loops
    g->stats.n_raw_edges = M;
    g->stats.n_self_loops = hc[1];
    TP_HIP(hipEventRecord(ev[1], s));

    // ---- phase 1: sort by pair
    const bool sorted_in_b = radix_sort_pairs(keyA.get(), valA.get(), keyB.get(), valB.get(), M, kb + dbit, s);
    uint64_t *skey = sorted_in_b ? keyB.get() : keyA.get();
    uint32_t *sval = sorted_in_b ? valB.get() : valA.get();
    uint64_t *fkey = sorted_in_b ? keyA.get() : keyB.get();  // free buffers
    uint32_t *fval = sorted_in_b ? valA.get() : valB.get();
    TP_HIP(hipEventRecord(ev[2], s));

    // ---- phase 2: dedup keeping the earliest time (and the directions)
    uint64_t m = 0;
    DArray<uint8_t> udir;
    if (directed) udir.reset(Mcap, s);
    {
        const size_t nt = std::max<size_t>(1, (Mv + kCompTile - 1) / kCompTile);
        DArray<uint64_t> toff(nt + 1, s);
        if (Mv) {
            k_dedup_count<<<(unsigned)nt, kB, 0, s>>>(skey, Mv, dbit, toff.get());
            TP_CHECK_LAUNCH();
        } else {
            TP_HIP(hipMemsetAsync(toff.get(), 0, sizeof(uint64_t), s));
        }
        scan_u64(toff.get(), toff.get(), nt, true, s);
        m = read_scalar(toff.get() + nt, s);
        if (Mv) {
            k_dedup_write<<<(unsigned)nt, kB, 0, s>>>(skey, sval, Mv, dbit, toff.get(), fkey, fval, udir.get());
            TP_CHECK_LAUNCH();
        }
    }
    uint64_t *ukey = fkey;
    uint32_t *uts = fval;
    g->m = m;
    g->stats.n_edges = m;
    TP_HIP(hipEventRecord(ev[3], s));

    // ---- phase 3: degree and the order <+
    DArray<uint32_t> rank(n, s);
    {
        DArray<uint32_t> deg(n, s);
        TP_HIP(hipMemsetAsync(deg.get(), 0, n * sizeof(uint32_t), s));
        if (m) {
            // the sorted (pre-dedup) pairs are no longer needed: their buffer
            // holds the two halves of the higher-end sort
            uint32_t *hiA = reinterpret_cast<uint32_t *>(skey), *hiB = hiA + Mcap;
            k_degree_low<<<grid_for(m, kB), kB, 0, s>>>(ukey, m, pc, deg.get(), hiA);
            TP_CHECK_LAUNCH();
            const bool hb2 = radix_sort_u32(hiA, hiB, m, nb, s);
            k_degree_runs<<<grid_for(m, kB), kB, 0, s>>>(hb2 ? hiB : hiA, m, deg.get());
            TP_CHECK_LAUNCH();
        }
        k_max<uint32_t><<<grid_for(n, kB), kB, 0, s>>>(deg.get(), n, c_dmax);
        TP_CHECK_LAUNCH();
        if (vlab) {
            k_max<uint8_t><<<grid_for(n, kB), kB, 0, s>>>(vlab, n, c_lab);
            TP_CHECK_LAUNCH();
        }
        unsigned long long mx[2];
        TP_HIP(hipMemcpyAsync(mx, c_dmax, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        TP_HIP(hipStreamSynchronize(s));
        g->stats.d_max = mx[0];
        g->stats.max_label = (uint32_t)mx[1];
        // sort keys (d(v), hash(v)) with the vertex as value
        DArray<uint64_t> rkeyA(n, s), rkeyB(n, s);
        DArray<uint32_t> rvalA(n, s), rvalB(n, s);
        const int gshift = nb + bits_for(mx[0]);
        const int rbits = gshift + (hb ? bits_for(hb->n_graphs - 1) : 0);
        if (rbits > 64) fail(TP_ERR_INVALID, "tripoll_build_batch: too many graphs and vertices for one order key");
        k_rank_keys<<<grid_for(n, kB), kB, 0, s>>>(deg.get(), n, nb, gshift, hb ? d_voff.get() : nullptr,
                                                   hb ? hb->n_graphs : 0u, el->tie_hash, rkeyA.get(), rvalA.get());
        TP_CHECK_LAUNCH();
        const bool rb = radix_sort_pairs(rkeyA.get(), rvalA.get(), rkeyB.get(), rvalB.get(), n, rbits, s);
        const uint64_t *skey = rb ? rkeyB.get() : rkeyA.get();
        g->perm = rb ? std::move(rvalB) : std::move(rvalA);
        g->rlab.reset(n, s);
        k_rank_scatter<<<grid_for(n, kB), kB, 0, s>>>(g->perm.get(), n, vlab, rank.get(), g->rlab.get());
        TP_CHECK_LAUNCH();
        if (hb) {
            g->n_graphs = hb->n_graphs;
            g->rank_gid.reset(n, s);
            k_rank_graph<<<grid_for(n, kB), kB, 0, s>>>(skey, n, gshift, g->rank_gid.get());
            TP_CHECK_LAUNCH();
        }
        {
            // bins 0 .. bin(d_max) are in use; 32 bounds per graph
            uint32_t top = 0;
            for (uint64_t d = mx[0]; d > 1 && top < 31; ++top) d = (d + 1) / 2;
            g->dbin_values = top + 1;
            const size_t nbins = (size_t)32 * (hb ? hb->n_graphs : 1u);
            g->dbin_rank.reset(nbins, s);
            fill_u32<<<grid_for(nbins, kB), kB, 0, s>>>(g->dbin_rank.get(), nbins, 0xffffffffu);
            TP_CHECK_LAUNCH();
            k_dbin_rank<<<grid_for(n, kB), kB, 0, s>>>(skey, n, nb, gshift, hb != nullptr, g->dbin_rank.get());
            TP_CHECK_LAUNCH();
        }
    }
    h_lab.release();
    TP_HIP(hipEventRecord(ev[4], s));

    // ---- phase 4: orient and sort by (source rank, target rank)
    DArray<uint32_t> dplus(n, s);
    TP_HIP(hipMemsetAsync(dplus.get(), 0, n * sizeof(uint32_t), s));
    if (m) {
        k_orient<<<grid_for(m, kB), kB, 0, s>>>(ukey, udir.get(), m, pc, rank.get(), skey);
        TP_CHECK_LAUNCH();
    }
    rank.release();
    udir.release();
    // keys from k_orient, values the dedup's times (same order); the
    // dedup's keys and the free value buffer take the other halves
    const bool ob = radix_sort_pairs(skey, uts, ukey, sval, m, kb + dbit2, s);
    uint64_t *okey = ob ? ukey : skey;
    uint32_t *ots = ob ? sval : uts;
    uint32_t *spare_val = ob ? uts : sval;
    TP_HIP(hipEventRecord(ev[5], s));

    // ---- phase 5: CSR with co-located metadata
    // col and ets carry kRowPad zeroed slots past the end: the survey loads a
    // whole wave of slots from any row start.  The sorted times are ets
    // itself: their buffer (sized for that pad) moves into the graph.
    g->col.reset(m + kRowPad, s);
    g->tlab.reset(std::max<uint64_t>(m, 1), s);
    g->ets = std::move(ots == valA.get() ? valA : valB);
    TP_HIP(hipMemsetAsync(g->col.get() + m, 0, kRowPad * sizeof(uint32_t), s));
    TP_HIP(hipMemsetAsync(g->ets.get() + m, 0, kRowPad * sizeof(uint32_t), s));
    if (directed) {
        g->directed = true;
        g->edir.reset(m + kRowPad * 4, s);
        TP_HIP(hipMemsetAsync(g->edir.get() + m, 0, kRowPad * 4, s));
    }
    uint32_t *srow = spare_val;
    if (m) {
        k_csr<<<grid_for(m, kB), kB, 0, s>>>(okey, m, pc, g->rlab.get(), g->col.get(), g->tlab.get(), srow,
                                             g->edir.get(), dplus.get());
        TP_CHECK_LAUNCH();
    }
    g->rowptr.reset((size_t)n + 1, s);
    scan_u32_to_u64(dplus.get(), g->rowptr.get(), n, s);
    dplus.release();
    k_row_stats<<<grid_for(n, kB), kB, 0, s>>>(g->rowptr.get(), n, c_wedge, c_dpmax);
    TP_CHECK_LAUNCH();
    if (g->dbin_rank.get()) {
        const size_t nbins = g->dbin_rank.n;
        g->dbin_slot.reset(nbins, s);
        k_dbin_slot<<<grid_for(nbins, 64), 64, 0, s>>>(g->dbin_rank.get(), g->rowptr.get(), nbins, g->dbin_slot.get());
        TP_CHECK_LAUNCH();
    }
    TP_HIP(hipEventRecord(ev[6], s));

    // ---- phase 6: in-edge index, a sort of the oriented edges by target
    {
        int kbits = std::max(1, bits_for(m));
        if (kbits + nb + 1 > 64) fail(TP_ERR_UNSUPPORTED, "tripoll_build: graph too large for the in-edge keys");
        g->kbits = (uint32_t)kbits;
        uint64_t *ikey = keyA.get(), *ikey_alt = keyB.get();
        // the payloads go to a buffer of their own (the sorted times became
        // ets); srow's buffer is free once the keys are written
        DArray<uint32_t> pay(std::max<uint64_t>(m, 1), s);
        uint32_t *ival = pay.get(), *ival_alt = srow;
        DArray<unsigned long long> kept(1, s);
        TP_HIP(hipMemsetAsync(kept.get(), 0, sizeof(unsigned long long), s));
        DArray<uint64_t> has_out;
        if (m) {
            has_out.reset((n + 63) / 64, s);
            k_has_out<<<grid_for(n, kB), kB, 0, s>>>(g->rowptr.get(), n, has_out.get());
            TP_CHECK_LAUNCH();
            k_in_keys<<<grid_for(m, kB), kB, 0, s>>>(srow, g->col.get(), g->rowptr.get(), has_out.get(),
                                                     g->rlab.get(), m, kbits, n, ikey, ival, kept.get());
            TP_CHECK_LAUNCH();
        }
        g->n_in = read_scalar(kept.get(), s);
        const bool alt = radix_sort_pairs(ikey, ival, ikey_alt, ival_alt, m, nb + 1, s, kbits);
        if (alt) {
            std::swap(ikey, ikey_alt);
            std::swap(ival, ival_alt);
        }
        // keep the sorted buffers as the index; the others go back to the pool
        DArray<uint64_t> &kk = (ikey == keyA.get()) ? keyA : keyB;
        DArray<uint32_t> &vv = (ival == pay.get()) ? pay : ((ival == valA.get()) ? valA : valB);
        g->inkey = std::move(kk);
        g->inpay = std::move(vv);
    }
    keyA.release();
    keyB.release();
    valA.release();
    valB.release();
    TP_HIP(hipEventRecord(ev[7], s));

    // ---- phase 7: work per target and the tile plan per class
    PlanCfg cfg{};
    for (int c = 0; c < kNumClasses; ++c) cfg.tile_records[c] = default_tile_records(c);
    g->stats.dplus_max = read_scalar(c_dpmax, s);  // the plan cuts huge targets' records
    plan_graph(g.get(), cfg, s);
    TP_HIP(hipEventRecord(ev[8], s));
    TP_HIP(hipStreamSynchronize(s));

    unsigned long long hs[8];
    TP_HIP(hipMemcpy(hs, counters.get(), 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    g->stats.n_vertices = n;
    g->stats.wedges = hs[4];
    g->stats.dplus_max = hs[5];
    // the survey packs a position in Adj+(q) into 22 bits; d+ <= sqrt(2m) keeps
    // this far away for any graph that fits in memory
    if (hs[5] >= (1ull << 22)) fail(TP_ERR_UNSUPPORTED, "tripoll_build: out-degree above 2^22 in the oriented graph");

    float total = 0.f;
    for (int i = 0; i < 8; ++i) {
        float t = 0.f;
        TP_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
        g->stats.phase_ms[i] = t;
        total += t;
    }
    g->stats.build_ms = total;
    g->stats.device_bytes = graph_bytes(g.get());
    *out = g.release();
}

extern "C" tp_status tripoll_build(const tp_edge_list *edges, void *stream, tp_graph **out)
{
    return guard([&] { build_impl(edges, (hipStream_t)stream, out); });
}

extern "C" tp_status tripoll_build_batch(const tp_batch_edges *be, void *stream, tp_graph **out)
{
    return guard([&] {
        if (!be || !out || !be->edge_offsets || !be->vertex_counts || be->n_graphs == 0)
            fail(TP_ERR_INVALID, "tripoll_build_batch: NULL argument or no graphs");
        HostBatch hb;
        hb.n_graphs = be->n_graphs;
        hb.eoff.assign(be->edge_offsets, be->edge_offsets + be->n_graphs + 1);
        hb.voff.resize(be->n_graphs + 1);
        uint64_t nv = 0;
        hb.voff[0] = 0;
        for (uint32_t i = 0; i < be->n_graphs; ++i) {
            if (hb.eoff[i + 1] < hb.eoff[i]) fail(TP_ERR_INVALID, "tripoll_build_batch: edge offsets decrease");
            nv += be->vertex_counts[i];
            if (nv >= 0xffffffffull) fail(TP_ERR_INVALID, "tripoll_build_batch: more than 2^32-2 vertices in all");
            hb.voff[i + 1] = (uint32_t)nv;
        }
        if (hb.eoff[0] != 0) fail(TP_ERR_INVALID, "tripoll_build_batch: edge_offsets[0] must be 0");
        if (nv == 0) fail(TP_ERR_INVALID, "tripoll_build_batch: no vertices");
        tp_edge_list el{};
        el.n_vertices = (uint32_t)nv;
        el.mem_space = be->mem_space;
        el.n_edges = hb.eoff[be->n_graphs];
        el.src = be->src;
        el.dst = be->dst;
        el.edge_time = be->edge_time;
        el.vertex_label = be->vertex_label;
        el.tie_hash = be->tie_hash;
        if (be->flags & ~TP_EDGES_DIRECTED) fail(TP_ERR_INVALID, "tripoll_build_batch: unknown flags");
        el.flags = be->flags;
        build_impl(&el, (hipStream_t)stream, out, &hb);
    });
}
