// tp_internal.hpp -- shared internals of libtripoll: error handling, the
// device memory pool, launch helpers and wave/block primitives for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "tripoll.h"

namespace tp {

// ---------------------------------------------------------------- errors

struct Error {
    tp_status status;
    std::string msg;
};

[[noreturn]] void fail(tp_status st, const std::string &msg);
void set_last_error(const std::string &msg);
void clear_last_error();

#define TP_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            (void)hipGetLastError();                                                      \
            ::tp::fail(e_ == hipErrorOutOfMemory ? TP_ERR_OOM : TP_ERR_DEVICE,            \
                       std::string(#call) + ": " + hipGetErrorString(e_));                \
        }                                                                                 \
    } while (0)

#define TP_CHECK_LAUNCH() TP_HIP(hipGetLastError())

// Run `body` and translate exceptions into a tp_status for the C ABI.
template <class F>
tp_status guard(F &&body)
{
    try {
        clear_last_error();
        body();
        return TP_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return TP_ERR_OOM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return TP_ERR_DEVICE;
    }
}

// ---------------------------------------------------------------- memory

// Caching device allocator: blocks obtained from hipMalloc are kept after
// release and handed out again for requests of similar size, so repeated
// builds do not pay for page mapping.  On an allocation failure the cache is
// returned to the driver and the request retried once.  Release is
// synchronous with respect to `stream` so a cached block is never handed out
// while a kernel may still touch it.
void *dev_alloc(size_t bytes);
void dev_release(void *p, hipStream_t stream);
void dev_trim();
size_t dev_cached_bytes();
size_t dev_live_bytes();   // bytes handed out and not yet released
void dev_fail_after(uint64_t n);  // fault injection: the n-th allocation from now fails (0: off)

// Owning device array, released into the cache.
template <class T>
struct DArray {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DArray() = default;
    DArray(size_t count, hipStream_t stream) { reset(count, stream); }
    DArray(const DArray &) = delete;
    DArray &operator=(const DArray &) = delete;
    DArray(DArray &&o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
    DArray &operator=(DArray &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p; n = o.n; s = o.s;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DArray() { release(); }
    void reset(size_t count, hipStream_t stream)
    {
        release();
        s = stream;
        n = count;
        p = count ? static_cast<T *>(dev_alloc(count * sizeof(T))) : nullptr;
    }
    void release()
    {
        if (p) dev_release(p, s);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    T *get() const { return p; }
};

// ---------------------------------------------------------------- launch

constexpr int kWave = 64;

// Claim counters of a survey launch: the last kClaimWords words of a result
// buffer's scratch and of a batch buffer.
constexpr uint32_t kClaimWords = 8;
constexpr uint32_t kRwClaim = TP_RW_SCRATCH + TP_RW_SCRATCH_WORDS - kClaimWords;
static_assert(TP_RW_SCRATCH_WORDS >= 8 + kClaimWords, "four counters, four class counts, the claim counters");
static_assert(TP_BATCH_SCRATCH_WORDS >= kClaimWords, "a batch buffer holds the claim counters");

inline unsigned grid_for(size_t n, int block, unsigned cap = 256u * 8u * 8u)
{
    size_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Timing helper: hipEvents recorded on a stream.
struct EventTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = nullptr;
    explicit EventTimer(hipStream_t stream) : s(stream)
    {
        TP_HIP(hipEventCreate(&a));
        TP_HIP(hipEventCreate(&b));
    }
    EventTimer(const EventTimer &) = delete;
    EventTimer &operator=(const EventTimer &) = delete;
    ~EventTimer()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start() { TP_HIP(hipEventRecord(a, s)); }
    void stop() { TP_HIP(hipEventRecord(b, s)); }
    float ms()
    {
        TP_HIP(hipEventSynchronize(b));
        float t = 0.f;
        TP_HIP(hipEventElapsedTime(&t, a, b));
        return t;
    }
};

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if ((int)lane_id() >= d) v += o;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        T o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Exclusive scan over a block of BLOCK threads; `tmp` is LDS of BLOCK/64 Ts.
// Returns the thread's exclusive prefix and writes the block total.
template <int BLOCK, class T>
__device__ __forceinline__ T block_excl_scan(T v, T *tmp, T &total)
{
    constexpr int NW = BLOCK / kWave;
    const int w = threadIdx.x / kWave;
    T incl = wave_incl_scan(v);
    if ((int)lane_id() == kWave - 1) tmp[w] = incl;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T x = tmp[i];
        if (i < w) base += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return base + incl - v;
}

// ---------------------------------------------------------------- primitives (prim.hip)

// Exclusive scan of n uint64 values (in may equal out).  Returns nothing; the
// total is written to out[n] if `with_total` (out must then hold n+1).
void scan_u64(const uint64_t *in, uint64_t *out, size_t n, bool with_total, hipStream_t s);
// Exclusive scan of n uint32 values into uint64 offsets (out holds n+1).
void scan_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on key bits [begin_bit,
// begin_bit + bits).  Sorts keys[0..n) with vals; alt buffers are scratch of
// the same size.  Returns true when the result ended in the alt buffers.
bool radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, size_t n,
                      int bits, hipStream_t s, int begin_bit = 0);
// The same for 32-bit keys alone.
bool radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, size_t n, int bits, hipStream_t s, int begin_bit = 0);

template <class T>
void fill(T *p, T v, size_t n, hipStream_t s);

inline int bits_for(uint64_t max_value)
{
    int b = 0;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

}  // namespace tp
