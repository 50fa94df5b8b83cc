// tpgen_dev.hip -- the seeded synthetic batch inputs, generated on the device.
//
// The same counter-based generator as tpgen.c (SplitMix64's output function
// over (seed, stream, index); Steele, Lea, Flood, OOPSLA 2014), written
// again for the GPU so that a batch of thousands of graphs can be produced
// in device memory directly instead of on the host and copied over.  Every
// value is a function of (seed, stream, index) only, so the device output is
// byte for byte that of tpgen.c (tested).  Like tpgen.c it holds none of the
// survey's arithmetic: it writes raw edge lists, times and labels only.
//
// A batch is described by one record per graph; the host cuts each graph's
// edges into chunks and every workgroup fills one chunk.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;
constexpr uint32_t kStreamEdge = 1, kStreamTs = 2, kStreamLabel = 3;

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_base(uint64_t seed, uint32_t stream)
{
    return mix64(seed + kGamma * ((uint64_t)stream + 1));
}

__device__ __forceinline__ uint64_t draw_at(uint64_t base, uint64_t index) { return mix64(base + kGamma * (index + 1)); }

}  // namespace

// One graph of a batch: recipe and placement.
struct tpgen_dev_graph {
    uint64_t seed;
    uint64_t edge_offset;   // first raw edge of the graph in the batch arrays
    uint64_t n_edges;
    uint64_t vertex_offset; // first label of the graph
    uint32_t kind;          // 0 R-MAT, 1 Erdos-Renyi
    uint32_t scale;         // n = 2^scale
    uint32_t ts_bits;       // times uniform on [0, 2^ts_bits)
    uint32_t n_labels;      // labels uniform on 0..n_labels-1
};

// A chunk of one graph's edges: [first, first + count) local edge indices.
struct tpgen_dev_chunk {
    uint32_t graph;
    uint32_t count;
    uint64_t first;
};

namespace {

// One workgroup per chunk.  R-MAT: level l of edge i takes the high half of
// draw i * ceil(scale / 2) + l / 2 for even l and the low half of that draw
// for odd l, quadrant (0,0), (0,1), (1,0), (1,1) below the cumulative
// thresholds, most significant bit first.  Erdos-Renyi: both endpoints from
// the two halves of draw i by the multiply-high map.  Times: the top ts_bits
// bits of draw i of the time stream.
__global__ void k_batch_edges(const tpgen_dev_graph *graphs, const tpgen_dev_chunk *chunks, uint32_t thr_a,
                              uint32_t thr_ab, uint32_t thr_abc, uint32_t *src, uint32_t *dst, uint32_t *ts)
{
    const tpgen_dev_chunk c = chunks[blockIdx.x];
    const tpgen_dev_graph g = graphs[c.graph];
    const uint64_t eb = stream_base(g.seed, kStreamEdge);
    const uint64_t tb = stream_base(g.seed, kStreamTs);
    const uint64_t per_edge = (g.scale + 1) / 2;
    const uint32_t n = 1u << g.scale;
    for (uint32_t j = threadIdx.x; j < c.count; j += blockDim.x) {
        const uint64_t i = c.first + j;
        uint32_t s = 0, d = 0;
        if (g.kind == 0) {
            uint64_t word = 0;
            for (uint32_t l = 0; l < g.scale; ++l) {
                uint32_t u;
                if ((l & 1u) == 0) {
                    word = draw_at(eb, i * per_edge + l / 2);
                    u = (uint32_t)(word >> 32);
                } else {
                    u = (uint32_t)word;
                }
                const uint32_t bit = 1u << (g.scale - 1 - l);
                if (u < thr_a) {
                } else if (u < thr_ab) {
                    d |= bit;
                } else if (u < thr_abc) {
                    s |= bit;
                } else {
                    s |= bit;
                    d |= bit;
                }
            }
        } else {
            const uint64_t w = draw_at(eb, i);
            s = (uint32_t)(((w >> 32) * (uint64_t)n) >> 32);
            d = (uint32_t)(((w & 0xffffffffull) * (uint64_t)n) >> 32);
        }
        const uint64_t at = g.edge_offset + i;
        src[at] = s;
        dst[at] = d;
        ts[at] = g.ts_bits == 0 ? 0u : (uint32_t)(draw_at(tb, i) >> (64 - g.ts_bits));
    }
}

// Labels: one workgroup per graph, label v = (high32(draw v) * L) >> 32.
__global__ void k_batch_labels(const tpgen_dev_graph *graphs, uint8_t *lab)
{
    const tpgen_dev_graph g = graphs[blockIdx.x];
    const uint64_t lb = stream_base(g.seed, kStreamLabel);
    const uint32_t n = 1u << g.scale;
    for (uint32_t v = threadIdx.x; v < n; v += blockDim.x)
        lab[g.vertex_offset + v] = (uint8_t)(((draw_at(lb, v) >> 32) * (uint64_t)g.n_labels) >> 32);
}

}  // namespace

// Fill the raw inputs of a batch in device memory.  `graphs` and `chunks`
// are device arrays (n_graphs and n_chunks records); src, dst, ts have room
// for every graph's edges and lab for every graph's vertices.  Enqueued on
// `stream`; returns 0, or a hipError_t of the launch.
extern "C" int tpgen_dev_batch(const tpgen_dev_graph *graphs, uint32_t n_graphs, const tpgen_dev_chunk *chunks,
                               uint32_t n_chunks, uint32_t thr_a, uint32_t thr_ab, uint32_t thr_abc, uint32_t *src,
                               uint32_t *dst, uint32_t *ts, uint8_t *lab, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (n_chunks) k_batch_edges<<<n_chunks, 256, 0, s>>>(graphs, chunks, thr_a, thr_ab, thr_abc, src, dst, ts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    if (n_graphs) k_batch_labels<<<n_graphs, 256, 0, s>>>(graphs, lab);
    return (int)hipGetLastError();
}
