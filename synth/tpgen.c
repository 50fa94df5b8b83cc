/*
 * tpgen.c -- seeded synthetic inputs for the triangle survey.
 *
 * This module only produces raw inputs (edge lists, edge timestamps, vertex
 * labels, per-graph batch parameters).  It holds none of the survey's
 * arithmetic: no cleaning, ordering, orientation or triangle logic lives here.
 * Both the CPU oracle tests and the GPU path read their inputs from it.
 *
 * Random numbers: a counter-based generator built from SplitMix64's output
 * function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  Draw i of stream s under seed S is
 *     base   = mix64(S + GAMMA * (s + 1))
 *     draw_i = mix64(base + GAMMA * (i + 1))
 * so every value depends only on (S, s, i): results are independent of the
 * number of threads and identical on every host.  All sampling below is
 * integer-only.
 *
 * Streams: 1 edges, 2 edge timestamps, 3 vertex labels, 4 burst parameters,
 * 5 per-graph batch parameters.
 */
#include <stdint.h>
#include <stddef.h>

#define GAMMA 0x9e3779b97f4a7c15ULL

enum { ST_EDGE = 1, ST_TS = 2, ST_LABEL = 3, ST_BURST = 4, ST_GPARAM = 5 };

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_base(uint64_t seed, uint32_t stream)
{
    return mix64(seed + GAMMA * ((uint64_t)stream + 1));
}

static inline uint64_t draw_at(uint64_t base, uint64_t index)
{
    return mix64(base + GAMMA * (index + 1));
}

uint64_t tpgen_draw(uint64_t seed, uint32_t stream, uint64_t index)
{
    return draw_at(stream_base(seed, stream), index);
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each edge descends `scale`
 * levels of the adjacency matrix, most significant bit first, choosing
 * quadrant (0,0),(0,1),(1,0),(1,1) with probabilities a, b, c, 1-a-b-c.
 * Level l of edge i uses a 32-bit uniform: the high half of draw
 * i*ceil(scale/2) + l/2 for even l, the low half for odd l.  thr_a, thr_ab,
 * thr_abc are the cumulative thresholds floor(p * 2^32).  No noise and no
 * vertex permutation.  Vertex count is 2^scale.
 */
void tpgen_rmat(uint64_t seed, uint32_t scale, uint64_t n_edges,
                uint32_t thr_a, uint32_t thr_ab, uint32_t thr_abc,
                uint32_t *src, uint32_t *dst)
{
    const uint64_t base = stream_base(seed, ST_EDGE);
    const uint64_t per_edge = (scale + 1) / 2;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)n_edges; ++i) {
        uint32_t s = 0, d = 0;
        uint64_t word = 0;
        for (uint32_t l = 0; l < scale; ++l) {
            uint32_t u;
            if ((l & 1) == 0) {
                word = draw_at(base, (uint64_t)i * per_edge + l / 2);
                u = (uint32_t)(word >> 32);
            } else {
                u = (uint32_t)word;
            }
            const uint32_t bit = scale - 1 - l;
            if (u < thr_a) {
                /* (0,0) */
            } else if (u < thr_ab) {
                d |= 1u << bit;
            } else if (u < thr_abc) {
                s |= 1u << bit;
            } else {
                s |= 1u << bit;
                d |= 1u << bit;
            }
        }
        src[i] = s;
        dst[i] = d;
    }
}

/* Erdos-Renyi G(n, M): M ordered pairs, each endpoint uniform on [0,n) by
 * the multiply-high map (u32 * n) >> 32 of one 32-bit half of a draw. */
void tpgen_er(uint64_t seed, uint32_t n, uint64_t n_edges, uint32_t *src, uint32_t *dst)
{
    const uint64_t base = stream_base(seed, ST_EDGE);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)n_edges; ++i) {
        const uint64_t w = draw_at(base, (uint64_t)i);
        src[i] = (uint32_t)(((w >> 32) * (uint64_t)n) >> 32);
        dst[i] = (uint32_t)(((w & 0xffffffffULL) * (uint64_t)n) >> 32);
    }
}

/* Timestamps uniform on [0, 2^bits): the top `bits` bits of draw i. */
void tpgen_ts_uniform(uint64_t seed, uint64_t count, uint32_t bits, uint32_t *ts)
{
    const uint64_t base = stream_base(seed, ST_TS);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)count; ++i)
        ts[i] = bits == 0 ? 0u : (uint32_t)(draw_at(base, (uint64_t)i) >> (64 - bits));
}

/*
 * Bursty timestamps: an equal-weight mixture of n_bursts Gaussian bursts over
 * [0, 2^31), clamped to [0, 2^31 - 1] and rounded down.
 *   centre_k = draw_burst(k) >> 33                   (uniform on [0, 2^31))
 *   sigma_k  = 2^(12 + draw_burst(n_bursts + k) mod 13)
 * Edge i uses draws 4i..4i+3 of the timestamp stream: burst k is the top
 * log2(n_bursts) bits of the fourth draw; the standard normal deviate is the
 * Irwin-Hall approximation (sum of twelve uniforms minus 6), formed in 16-bit
 * fixed point from the twelve 16-bit halves of the first three draws.
 * n_bursts must be a power of two <= 64.
 */
void tpgen_ts_bursty(uint64_t seed, uint64_t count, uint32_t n_bursts, uint32_t *ts)
{
    uint64_t centre[64];
    uint32_t expo[64];
    const uint64_t bb = stream_base(seed, ST_BURST);
    uint32_t kbits = 0;
    while ((1u << kbits) < n_bursts) ++kbits;
    for (uint32_t k = 0; k < n_bursts; ++k) {
        centre[k] = draw_at(bb, k) >> 33;
        expo[k] = 12u + (uint32_t)(draw_at(bb, n_bursts + k) % 13u);
    }
    const uint64_t base = stream_base(seed, ST_TS);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)count; ++i) {
        int64_t sum = 0;
        for (int j = 0; j < 3; ++j) {
            const uint64_t w = draw_at(base, 4 * (uint64_t)i + j);
            sum += (int64_t)(w & 0xffff) + (int64_t)((w >> 16) & 0xffff) +
                   (int64_t)((w >> 32) & 0xffff) + (int64_t)(w >> 48);
        }
        const uint64_t w3 = draw_at(base, 4 * (uint64_t)i + 3);
        const uint32_t k = kbits == 0 ? 0u : (uint32_t)(w3 >> (64 - kbits));
        const int64_t z = sum - 6 * 65536;           /* N(0,1) in units of 2^-16 */
        const int64_t off = (z * ((int64_t)1 << expo[k])) >> 16;
        int64_t v = (int64_t)centre[k] + off;
        if (v < 0) v = 0;
        if (v > 0x7fffffffLL) v = 0x7fffffffLL;
        ts[i] = (uint32_t)v;
    }
}

/* Labels uniform on 0..L-1: (high32(draw_v) * L) >> 32. */
void tpgen_labels_uniform(uint64_t seed, uint32_t n, uint32_t L, uint8_t *lab)
{
    const uint64_t base = stream_base(seed, ST_LABEL);
    int64_t v;
#pragma omp parallel for schedule(static)
    for (v = 0; v < (int64_t)n; ++v)
        lab[v] = (uint8_t)(((draw_at(base, (uint64_t)v) >> 32) * (uint64_t)L) >> 32);
}

/* Labels from an integer CDF: label = least k with high32(draw_v) < thr[k];
 * thr has L-1 entries (the last class takes the rest). */
void tpgen_labels_cdf(uint64_t seed, uint32_t n, const uint32_t *thr, uint32_t L, uint8_t *lab)
{
    const uint64_t base = stream_base(seed, ST_LABEL);
    int64_t v;
#pragma omp parallel for schedule(static)
    for (v = 0; v < (int64_t)n; ++v) {
        const uint32_t u = (uint32_t)(draw_at(base, (uint64_t)v) >> 32);
        uint32_t k = 0;
        while (k + 1 < L && u >= thr[k]) ++k;
        lab[v] = (uint8_t)k;
    }
}

/* Per-graph parameters of a batch: graph g gets its own seed and, from draws
 * 0..2 of that seed's parameter stream, kind (0 R-MAT, 1 Erdos-Renyi),
 * scale in [scale_lo, scale_hi] and edge factor in [ef_lo, ef_hi]. */
void tpgen_batch_params(uint64_t master, uint32_t g,
                        uint32_t scale_lo, uint32_t scale_hi, uint32_t ef_lo, uint32_t ef_hi,
                        uint64_t *seed_g, uint32_t *kind, uint32_t *scale, uint32_t *ef)
{
    const uint64_t sg = tpgen_draw(master, ST_GPARAM, g);
    const uint64_t b = stream_base(sg, ST_GPARAM);
    *seed_g = sg;
    *kind = (uint32_t)(draw_at(b, 0) >> 63);
    *scale = scale_lo + (uint32_t)(draw_at(b, 1) % (uint64_t)(scale_hi - scale_lo + 1));
    *ef = ef_lo + (uint32_t)(draw_at(b, 2) % (uint64_t)(ef_hi - ef_lo + 1));
}
