// prim.hip -- library runtime pieces and device primitives for gfx950:
// per-thread error state, the caching device allocator, exclusive scans and
// a stable LSD radix sort of (uint64 key, uint32 value) pairs.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>

#include "tp_internal.hpp"

namespace tp {

// ================================================================ errors

static thread_local std::string g_last_error;

void fail(tp_status st, const std::string &msg) { throw Error{st, msg}; }
void set_last_error(const std::string &msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }
const char *last_error_cstr() { return g_last_error.c_str(); }

// ================================================================ allocator

namespace {

struct Pool {
    std::mutex mu;
    std::multimap<size_t, void *> free_blocks;        // size -> block
    std::unordered_map<void *, size_t> live;          // block -> size
    size_t cached = 0;
};

Pool &pool_for_current_device()
{
    static std::mutex m;
    static std::map<int, Pool *> pools;
    int dev = 0;
    TP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(m);
    Pool *&p = pools[dev];
    if (!p) p = new Pool();  // lives until process exit
    return *p;
}

size_t round_size(size_t bytes)
{
    const size_t small = 512, big = size_t(2) << 20;
    return bytes < big ? (bytes + small - 1) / small * small : (bytes + big - 1) / big * big;
}

void trim_locked(Pool &p)
{
    for (auto &kv : p.free_blocks) (void)hipFree(kv.second);
    p.free_blocks.clear();
    p.cached = 0;
}

// Fault injection: when non-zero, the allocation that brings it to zero
// fails as if the device were out of memory.
std::atomic<uint64_t> g_fail_countdown{0};

}  // namespace

void dev_fail_after(uint64_t n) { g_fail_countdown.store(n); }

void *dev_alloc(size_t bytes)
{
    for (uint64_t c = g_fail_countdown.load(); c;) {
        if (g_fail_countdown.compare_exchange_weak(c, c - 1)) {
            if (c == 1) fail(TP_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed (injected)");
            break;
        }
    }
    Pool &p = pool_for_current_device();
    const size_t sz = round_size(bytes ? bytes : 1);
    std::lock_guard<std::mutex> lk(p.mu);
    auto it = p.free_blocks.lower_bound(sz);
    // reuse a cached block when it is not much larger than the request
    if (it != p.free_blocks.end() && it->first <= sz + sz / 4 + (size_t(8) << 20)) {
        void *ptr = it->second;
        p.live[ptr] = it->first;
        p.cached -= it->first;
        p.free_blocks.erase(it);
        return ptr;
    }
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, sz);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        trim_locked(p);
        e = hipMalloc(&ptr, sz);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? TP_ERR_OOM : TP_ERR_DEVICE,
             "device allocation of " + std::to_string(sz) + " bytes failed: " + hipGetErrorString(e));
    }
    p.live[ptr] = sz;
    return ptr;
}

void dev_release(void *ptr, hipStream_t stream)
{
    if (!ptr) return;
    // the block may still be in use by work on `stream`
    (void)hipStreamSynchronize(stream);
    Pool &p = pool_for_current_device();
    std::lock_guard<std::mutex> lk(p.mu);
    auto it = p.live.find(ptr);
    if (it == p.live.end()) return;
    p.free_blocks.emplace(it->second, ptr);
    p.cached += it->second;
    p.live.erase(it);
}

void dev_trim()
{
    Pool &p = pool_for_current_device();
    std::lock_guard<std::mutex> lk(p.mu);
    trim_locked(p);
}

size_t dev_cached_bytes()
{
    Pool &p = pool_for_current_device();
    std::lock_guard<std::mutex> lk(p.mu);
    return p.cached;
}

size_t dev_live_bytes()
{
    Pool &p = pool_for_current_device();
    std::lock_guard<std::mutex> lk(p.mu);
    size_t b = 0;
    for (const auto &kv : p.live) b += kv.second;
    return b;
}

// ================================================================ fill

template <class T>
__global__ void fill_kernel(T *p, T v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
void fill(T *p, T v, size_t n, hipStream_t s)
{
    if (!n) return;
    fill_kernel<T><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    TP_CHECK_LAUNCH();
}
template void fill<uint32_t>(uint32_t *, uint32_t, size_t, hipStream_t);
template void fill<uint64_t>(uint64_t *, uint64_t, size_t, hipStream_t);
template void fill<uint8_t>(uint8_t *, uint8_t, size_t, hipStream_t);

// ================================================================ scan

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr size_t kScanTile = (size_t)kScanBlock * kScanItems;

template <class Tin>
__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const Tin *in, uint64_t *partial, size_t n)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    const size_t base = blockIdx.x * kScanTile;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const size_t i = base + (size_t)j * kScanBlock + threadIdx.x;
        if (i < n) s += (uint64_t)in[i];
    }
    s = wave_sum(s);
    if (lane_id() == 0) tmp[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) t += tmp[w];
        partial[blockIdx.x] = t;
    }
}

// Each thread owns kScanItems consecutive elements.
template <class Tin>
__global__ __launch_bounds__(kScanBlock) void scan_block_kernel(const Tin *in, uint64_t *out, size_t n,
                                                                 const uint64_t *partial, uint64_t *total_out)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    const size_t base = blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const size_t i = base + j;
        v[j] = i < n ? (uint64_t)in[i] : 0;
        s += v[j];
    }
    uint64_t tot;
    uint64_t pre = block_excl_scan<kScanBlock>(s, tmp, tot);
    pre += partial ? partial[blockIdx.x] : 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const size_t i = base + j;
        if (i < n) out[i] = pre;
        pre += v[j];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1) *total_out = pre;
}

template <class Tin>
void scan_impl(const Tin *in, uint64_t *out, size_t n, uint64_t *total_out, hipStream_t s)
{
    if (n == 0) {
        if (total_out) TP_HIP(hipMemsetAsync(total_out, 0, sizeof(uint64_t), s));
        return;
    }
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        scan_block_kernel<Tin><<<1, kScanBlock, 0, s>>>(in, out, n, nullptr, total_out);
        TP_CHECK_LAUNCH();
        return;
    }
    DArray<uint64_t> partial(nb, s);
    scan_reduce_kernel<Tin><<<(unsigned)nb, kScanBlock, 0, s>>>(in, partial.get(), n);
    TP_CHECK_LAUNCH();
    scan_impl<uint64_t>(partial.get(), partial.get(), nb, nullptr, s);
    scan_block_kernel<Tin><<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, n, partial.get(), total_out);
    TP_CHECK_LAUNCH();
}

}  // namespace

void scan_u64(const uint64_t *in, uint64_t *out, size_t n, bool with_total, hipStream_t s)
{
    scan_impl<uint64_t>(in, out, n, with_total ? out + n : nullptr, s);
}

void scan_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n, hipStream_t s)
{
    scan_impl<uint32_t>(in, out, n, out + n, s);
}

// ================================================================ radix sort
//
// Reduce-then-scan LSD radix sort, 9-bit digits (52-bit pair keys take 6
// passes; 8-bit digits took 7 and were slower overall, 10-bit digits write
// runs too short to coalesce), except that a sort takes some 10-bit digits
// where they save a pass (56-bit keys: 6 passes, two of them 10-bit, not 7).
// A fixed number of blocks each own a contiguous chunk of tiles (4096
// keys).  Per pass:
//   1. upsweep: digit histogram of each block's chunk -> hist[digit][block]
//   2. exclusive scan of hist (digit-major), giving each (digit, block) its
//      first output position
//   3. downsweep: per tile, each wave ranks its quarter of the tile stably
//      with ballot-based digit matching; the tile is reordered in LDS by
//      digit and written out in digit runs, so stores are contiguous.

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortRounds = 16;                           // keys per lane
constexpr int kSortTile = kSortBlock * kSortRounds;       // 4096
constexpr int kMaxRadixBits = 10;
constexpr unsigned kMaxSortBlocks = 2048;

template <int RB>
__device__ __forceinline__ unsigned digit_of(uint64_t k, int shift)
{
    return (unsigned)(k >> shift) & ((1u << RB) - 1);
}

template <class K, int RB>
__global__ __launch_bounds__(kSortBlock) void radix_upsweep(const K *keys, size_t n, int shift,
                                                            size_t tiles_per_block, uint64_t *hist)
{
    constexpr int kRadix = 1 << RB;
    __shared__ unsigned cnt[kRadix];
    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) cnt[d] = 0;
    __syncthreads();
    const size_t t0 = blockIdx.x * tiles_per_block;
    const size_t lo = t0 * kSortTile;
    const size_t hi = std::min(n, (t0 + tiles_per_block) * kSortTile);
    for (size_t i = lo + threadIdx.x; i < hi; i += kSortBlock) atomicAdd(&cnt[digit_of<RB>(keys[i], shift)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) hist[(size_t)d * gridDim.x + blockIdx.x] = cnt[d];
}

// K: uint64_t or uint32_t keys; VALS: whether 32-bit values travel with
// them; RB: bits of the digit.
template <class K, bool VALS, int RB>
// (two blocks of 4 waves per compute unit: 10-bit digits with values need
// all of 256 registers and 80 KB of LDS for it)
__global__ __launch_bounds__(kSortBlock, 2) void radix_downsweep(const K *keys_in, const uint32_t *vals_in,
                                                              K *keys_out, uint32_t *vals_out, size_t n,
                                                              int shift, size_t tiles_per_block,
                                                              const uint64_t *offsets)
{
    constexpr int kRadix = 1 << RB;
    constexpr int kDigitsPerThread = kRadix / kSortBlock;
    __shared__ K skey[kSortTile];
    __shared__ uint32_t sval[VALS ? kSortTile : 1];
    __shared__ unsigned wcnt[kSortWaves][kRadix];  // per-wave running count, then per-wave base
    __shared__ unsigned tstart[kRadix];
    __shared__ uint64_t grun[kRadix];              // next output position of each digit
    __shared__ unsigned scan_tmp[kSortWaves];

    const int w = threadIdx.x / kWave;
    const unsigned lane = lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
        grun[d] = offsets[(size_t)d * gridDim.x + blockIdx.x];
        for (int i = 0; i < kSortWaves; ++i) wcnt[i][d] = 0;
    }
    __syncthreads();

    const size_t t0 = blockIdx.x * tiles_per_block;
    // the keys and values of the next tile are requested while this one is
    // ranked and written, so that the loads overlap the tile's work
    K kn[kSortRounds];
    uint32_t vn[kSortRounds];
    auto load_tile = [&](size_t t) {
        const size_t wl = t * kSortTile + (size_t)w * (kSortTile / kSortWaves);
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const size_t i = wl + (size_t)r * kWave + lane;
            kn[r] = i < n ? keys_in[i] : 0;
            vn[r] = (VALS && i < n) ? vals_in[i] : 0;
        }
    };
    if (t0 * kSortTile < n) load_tile(t0);
    for (size_t t = t0; t < t0 + tiles_per_block; ++t) {
        const size_t tile_lo = t * kSortTile;
        if (tile_lo >= n) break;
        const size_t wave_lo = tile_lo + (size_t)w * (kSortTile / kSortWaves);

        K k[kSortRounds];
        uint32_t v[kSortRounds];
        unsigned rnk[kSortRounds];
        unsigned dg[kSortRounds];
        bool ok[kSortRounds];
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            const size_t i = wave_lo + (size_t)r * kWave + lane;
            ok[r] = i < n;
            k[r] = kn[r];
            v[r] = vn[r];
            dg[r] = digit_of<RB>(k[r], shift);
        }
        if (t + 1 < t0 + tiles_per_block && (t + 1) * kSortTile < n) load_tile(t + 1);
        // stable rank of every key among equal digits of this wave's quarter
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            uint64_t peers = __ballot(ok[r]);
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const bool bit = (dg[r] >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            unsigned before = 0;
            if (ok[r]) {
                before = wcnt[w][dg[r]];
                rnk[r] = before + (unsigned)__popcll(peers & lt_mask);
            }
            // the lowest lane of each digit group advances the running count;
            // same-wave LDS accesses are performed in program order
            if (ok[r] && (peers & lt_mask) == 0) wcnt[w][dg[r]] = before + (unsigned)__popcll(peers);
        }
        __syncthreads();
        // per-digit totals, wave bases and tile starts
        {
            unsigned loc[kDigitsPerThread];
            unsigned sum = 0;
#pragma unroll
            for (int j = 0; j < kDigitsPerThread; ++j) {
                const unsigned d = threadIdx.x * kDigitsPerThread + j;
                unsigned tot = 0;
                for (int i = 0; i < kSortWaves; ++i) {
                    const unsigned c = wcnt[i][d];
                    wcnt[i][d] = tot;
                    tot += c;
                }
                loc[j] = sum;
                sum += tot;
            }
            unsigned total;
            const unsigned base = block_excl_scan<kSortBlock>(sum, scan_tmp, total);
#pragma unroll
            for (int j = 0; j < kDigitsPerThread; ++j) tstart[threadIdx.x * kDigitsPerThread + j] = base + loc[j];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortRounds; ++r) {
            if (ok[r]) {
                const unsigned pos = tstart[dg[r]] + wcnt[w][dg[r]] + rnk[r];
                skey[pos] = k[r];
                if (VALS) sval[pos] = v[r];
            }
        }
        __syncthreads();
        const unsigned valid = (unsigned)std::min<size_t>(kSortTile, n - tile_lo);
        for (unsigned i = threadIdx.x; i < valid; i += kSortBlock) {
            const K key = skey[i];
            const unsigned d = digit_of<RB>(key, shift);
            const uint64_t dst = grun[d] + (i - tstart[d]);
            keys_out[dst] = key;
            if (VALS) vals_out[dst] = sval[i];
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
            // the digit's keys in this tile: up to the next digit's start
            grun[d] += (d + 1 < kRadix ? tstart[d + 1] : valid) - tstart[d];
            for (int i = 0; i < kSortWaves; ++i) wcnt[i][d] = 0;
        }
        __syncthreads();
    }
}

// One pass over digit [shift, shift + RB): histograms, their scan, the
// stable scatter (values travel when vi is set).
template <class K, int RB>
void sort_pass(const K *ki, const uint32_t *vi, K *ko, uint32_t *vo, size_t n, int shift, unsigned nb, size_t tpb,
               uint64_t *hist, hipStream_t s)
{
    radix_upsweep<K, RB><<<nb, kSortBlock, 0, s>>>(ki, n, shift, tpb, hist);
    TP_CHECK_LAUNCH();
    scan_u64(hist, hist, (size_t)(1u << RB) * nb, false, s);
    if (vi)
        radix_downsweep<K, true, RB><<<nb, kSortBlock, 0, s>>>(ki, vi, ko, vo, n, shift, tpb, hist);
    else
        radix_downsweep<K, false, RB><<<nb, kSortBlock, 0, s>>>(ki, nullptr, ko, nullptr, n, shift, tpb, hist);
    TP_CHECK_LAUNCH();
}

template <class K>
bool radix_sort(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, size_t n, int bits, hipStream_t s,
                int begin_bit)
{
    if (n <= 1 || bits <= 0) return false;
    const size_t tiles = (n + kSortTile - 1) / kSortTile;
    const unsigned nb = (unsigned)std::min<size_t>(tiles, kMaxSortBlocks);
    const size_t tpb = (tiles + nb - 1) / nb;
    DArray<uint64_t> hist((size_t)(1u << kMaxRadixBits) * nb, s);
    // 9-bit digits, or as few 10-bit ones as cover `bits` in one pass less
    const int p9 = (bits + 8) / 9, p10 = (bits + 9) / 10;
    const int passes = std::min(p9, p10);
    const int n10 = passes < p9 ? bits - 9 * passes : 0;
    bool in_alt = false;
    int shift = begin_bit;
    for (int pass = 0; pass < passes; ++pass) {
        const K *ki = in_alt ? keys_alt : keys;
        const uint32_t *vi = in_alt ? vals_alt : vals;
        K *ko = in_alt ? keys : keys_alt;
        uint32_t *vo = in_alt ? vals : vals_alt;
        if (pass < n10) sort_pass<K, 10>(ki, vi, ko, vo, n, shift, nb, tpb, hist.get(), s);
        else sort_pass<K, 9>(ki, vi, ko, vo, n, shift, nb, tpb, hist.get(), s);
        shift += pass < n10 ? 10 : 9;
        in_alt = !in_alt;
    }
    return in_alt;
}

}  // namespace

bool radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, size_t n, int bits,
                      hipStream_t s, int begin_bit)
{
    return radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, s, begin_bit);
}

bool radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, size_t n, int bits, hipStream_t s, int begin_bit)
{
    return radix_sort<uint32_t>(keys, nullptr, keys_alt, nullptr, n, bits, s, begin_bit);
}

}  // namespace tp
