/*
 * oracle.c -- plain CPU reference of the metadata triangle survey.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests and the benchmark's CPU baseline can
 * check the GPU results.  It shares no code, header or constant with the GPU
 * path.
 *
 * What it computes follows the paper (Steil et al., "TriPoll: Computing
 * Surveys of Triangles in Massive-Scale Temporal Graphs with Metadata"):
 *
 *   - Preliminaries: the input is an undirected graph; d(v) = |Adj(v)|; a
 *     triangle is three vertices pairwise joined by edges; meta(v) and
 *     meta(u,v) = meta(v,u) decorate vertices and edges; vertices are ordered
 *     by degree with a deterministic tie-break, and each undirected edge is
 *     oriented from the lower to the higher vertex (the DODGr), so that every
 *     triangle p < q < r is found exactly once, from its pivot p.
 *   - Datasets subsection: a multigraph is reduced by keeping the
 *     chronologically first edge between two vertices; self-loops carry no
 *     triangle.
 *   - Algorithm 1 (Push-Only survey): for every p and every q in Adj+(p),
 *     intersect the rest of Adj+(p) with Adj+(q) by a merge of two sorted
 *     lists and hand the six metadata items of each triangle to a callback.
 *   - Algorithms 2 and 4: the counting callback and the closure-time callback
 *     (t1 <= t2 <= t3 the sorted edge timestamps; close = ceil(log2(t3 - t1)),
 *     open = ceil(log2(t2 - t1))).
 *   - Algorithm 3: among triangles whose three vertex labels are pairwise
 *     distinct, the distribution of the largest edge metadata (here the edge
 *     time t3).  The paper counts exact values in a counting set; here the
 *     count is kept per 2^shift-wide range of t3 (bin t3 >> shift, the last
 *     of 1024 bins taking everything above), which is the exact counting set
 *     whenever every t3 >> shift is below 1024.
 *   - Local participation (Introduction; Triangle Counting subsection): per
 *     vertex and per edge, the number of triangles that contain it (the
 *     counters of clustering coefficients and truss decomposition), under
 *     the same prefilters as the surveys.
 *   - Directed graphs (the remark closing the Preliminaries' storage
 *     discussion: the oriented graph serves directed inputs too, each edge
 *     keeping two bits of its original direction): a census of the
 *     directed triangle types.  Each vertex pair keeps which directions
 *     occur among its raw copies; a triangle is then one of seven types of
 *     three connected pairs, named as in the triad census: 030T (three
 *     one-way arcs, no cycle), 030C (a directed 3-cycle), 120D, 120U, 120C
 *     (one mutual pair; the third vertex sends both of its arcs, receives
 *     both, or sends one and receives one), 210 (two mutual pairs) and 300
 *     (three mutual pairs).
 *   - Metadata-overhead experiment of the evaluation (vertex degree as the
 *     metadata): counts of the triple (ceil(log2 d(p)), ceil(log2 d(q)),
 *     ceil(log2 d(r))) over all triangles, p, q, r in the degree order.
 *     Because the three are in degree order the triple is non-decreasing, so
 *     it is the sorted triple of the three vertices' values and is counted by
 *     its multiset index, like the label table.
 *
 * The oracle orders vertices by (degree, original id), i.e. the paper's order
 * with the identity as tie-break, and keeps every out-list sorted by original
 * id; since every out-neighbour of v is above v in the order, the full merge
 * of Adj+(p) and Adj+(q) finds exactly the closing vertices r of Algorithm 1.
 *
 * Integer readings of the callbacks (the paper states them with real log2):
 *   bin(D)  = 0 for D <= 1, else min(31, ceil(log2 D)) computed exactly.
 *   msidx   = rank of the label multiset a <= b <= c in colex order:
 *             C(c+2,3) + C(b+1,2) + a.
 * Every counter is an unsigned 64-bit integer, so results do not depend on the
 * enumeration order and are exact.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OUT_COUNT 1u
#define ORC_OUT_CLOSE_HIST 2u
#define ORC_OUT_LABEL_TABLE 4u
#define ORC_OUT_SPREAD 8u
#define ORC_OUT_OPEN_CLOSE 16u
#define ORC_OUT_MAX_EDGE 32u
#define ORC_OUT_DEGREE_TABLE 64u
#define ORC_OUT_DIRECTED 128u

#define ORC_FILT_WINDOW 1u
#define ORC_FILT_LABEL_MASK 2u

#define ORC_MAX_LABELS 16
#define ORC_TABLE_MAX 816 /* C(16+2, 3) */
#define ORC_MAX_EDGE_BINS 1024
#define ORC_DEGREE_MAX 5984 /* C(32+2, 3): degree bins 0..31 */

typedef struct {
    uint32_t outputs;
    uint32_t filters;
    uint32_t n_labels;
    uint32_t max_edge_shift; /* Algorithm 3 bins: t3 >> max_edge_shift */
    uint64_t spread_lt;   /* spread counter: max(t) - min(t) < spread_lt */
    uint64_t t_lo, t_hi;  /* window filter: all three t in [t_lo, t_hi] */
    uint64_t label_mask[(ORC_TABLE_MAX + 63) / 64];
} orc_spec;

typedef struct {
    uint64_t triangles;
    uint64_t spread_count;
    uint64_t wedges;
    uint64_t close_hist[32];
    uint64_t label_table[ORC_TABLE_MAX];
    uint64_t open_close[32 * 32];
    uint64_t max_edge[ORC_MAX_EDGE_BINS];
    uint64_t degree_table[ORC_DEGREE_MAX];
    uint64_t directed[7]; /* 030T, 030C, 120D, 120U, 120C, 210, 300 */
} orc_result;

/* ------------------------------------------------------------------------ */
/* Callback arithmetic                                                       */
/* ------------------------------------------------------------------------ */

/* ceil(log2(D)) for D >= 2 without floating point: the number of bits of
 * D - 1.  D = 0 and D = 1 share bin 0; saturate at 31. */
uint32_t oracle_bin(uint64_t d)
{
    if (d <= 1)
        return 0;
    uint64_t x = d - 1;
    uint32_t bits = 0;
    while (x) {
        ++bits;
        x >>= 1;
    }
    return bits > 31 ? 31 : bits;
}

static uint64_t choose(uint64_t n, uint64_t k)
{
    if (k > n)
        return 0;
    uint64_t r = 1;
    for (uint64_t i = 1; i <= k; ++i)
        r = r * (n - k + i) / i;
    return r;
}

/* Colex rank of the multiset {a <= b <= c}. */
uint32_t oracle_msidx(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return (uint32_t)(choose(c + 2, 3) + choose(b + 1, 2) + a);
}

/* The prefilters: all three times in the closed window, and the label
 * multiset's bit set in the mask. */
static int passes(const orc_spec *sp, uint32_t t_pq, uint32_t t_pr, uint32_t t_qr,
                  uint8_t l_p, uint8_t l_q, uint8_t l_r)
{
    if (sp->filters & ORC_FILT_WINDOW) {
        if (t_pq < sp->t_lo || t_pq > sp->t_hi) return 0;
        if (t_pr < sp->t_lo || t_pr > sp->t_hi) return 0;
        if (t_qr < sp->t_lo || t_qr > sp->t_hi) return 0;
    }
    if (sp->filters & ORC_FILT_LABEL_MASK) {
        const uint32_t idx = oracle_msidx(l_p, l_q, l_r);
        if (!((sp->label_mask[idx / 64] >> (idx % 64)) & 1u)) return 0;
    }
    return 1;
}

/* Type of a directed triangle on vertices 0, 1, 2 given each pair's
 * directions: d01 has bit 0 for the arc 0 -> 1 and bit 1 for 1 -> 0, and
 * likewise d02 (0 -> 2, 2 -> 0) and d12 (1 -> 2, 2 -> 1).  Every pair has at
 * least one arc. */
uint32_t oracle_directed_type(uint32_t d01, uint32_t d02, uint32_t d12)
{
    int arc[3][3] = {{0}};
    arc[0][1] = d01 & 1; arc[1][0] = (d01 >> 1) & 1;
    arc[0][2] = d02 & 1; arc[2][0] = (d02 >> 1) & 1;
    arc[1][2] = d12 & 1; arc[2][1] = (d12 >> 1) & 1;
    int mutual = 0, x = -1, y = -1;
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (arc[i][j] && arc[j][i]) { ++mutual; x = i; y = j; }
    if (mutual == 3) return 6;
    if (mutual == 2) return 5;
    if (mutual == 1) {
        const int z = 3 - x - y;  /* the vertex outside the mutual pair */
        const int out = arc[z][x] + arc[z][y], in = arc[x][z] + arc[y][z];
        if (out == 2) return 2;  /* 120D */
        if (in == 2) return 3;   /* 120U */
        return 4;                /* 120C */
    }
    /* three one-way arcs: a cycle when every vertex sends exactly one */
    for (int i = 0; i < 3; ++i)
        if (arc[i][0] + arc[i][1] + arc[i][2] != 1) return 0;  /* 030T */
    return 1;                                                 /* 030C */
}

static void callback(const orc_spec *sp, orc_result *acc,
                     uint32_t t_pq, uint32_t t_pr, uint32_t t_qr,
                     uint8_t l_p, uint8_t l_q, uint8_t l_r,
                     uint64_t d_p, uint64_t d_q, uint64_t d_r, uint32_t type)
{
    if (!passes(sp, t_pq, t_pr, t_qr, l_p, l_q, l_r)) return;
    uint32_t idx = 0;
    if (sp->outputs & ORC_OUT_LABEL_TABLE)
        idx = oracle_msidx(l_p, l_q, l_r);
    /* sorted timestamps t1 <= t2 <= t3 */
    uint32_t t1 = t_pq, t2 = t_pr, t3 = t_qr, t;
    if (t1 > t2) { t = t1; t1 = t2; t2 = t; }
    if (t2 > t3) { t = t2; t2 = t3; t3 = t; }
    if (t1 > t2) { t = t1; t1 = t2; t2 = t; }
    const uint64_t close = (uint64_t)t3 - t1;
    const uint64_t open = (uint64_t)t2 - t1;

    acc->triangles += 1;
    if (sp->outputs & ORC_OUT_CLOSE_HIST)
        acc->close_hist[oracle_bin(close)] += 1;
    if (sp->outputs & ORC_OUT_LABEL_TABLE)
        acc->label_table[idx] += 1;
    if (sp->outputs & ORC_OUT_SPREAD)
        acc->spread_count += (close < sp->spread_lt) ? 1u : 0u;
    if (sp->outputs & ORC_OUT_OPEN_CLOSE)
        acc->open_close[oracle_bin(open) * 32 + oracle_bin(close)] += 1;
    if ((sp->outputs & ORC_OUT_MAX_EDGE) && l_p != l_q && l_q != l_r && l_p != l_r) {
        /* the largest of the three edge times, t3, in its range of 2^shift */
        uint64_t b = (uint64_t)t3 >> sp->max_edge_shift;
        if (b > ORC_MAX_EDGE_BINS - 1) b = ORC_MAX_EDGE_BINS - 1;
        acc->max_edge[b] += 1;
    }
    if (sp->outputs & ORC_OUT_DEGREE_TABLE)
        acc->degree_table[oracle_msidx(oracle_bin(d_p), oracle_bin(d_q), oracle_bin(d_r))] += 1;
    if (sp->outputs & ORC_OUT_DIRECTED)
        acc->directed[type] += 1;
}

/* Directions of the pair {x, y} as seen from x -> y, given the bits of the
 * cleaned pair (bit 0: lower id -> higher id, bit 1: higher -> lower). */
static uint32_t dir_from(uint32_t x, uint32_t y, uint32_t bits)
{
    return x < y ? bits : (((bits & 1u) << 1) | (bits >> 1));
}

/* ------------------------------------------------------------------------ */
/* Cleaning: self-loops dropped, each undirected pair once, earliest time.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key; /* (min << 32) | max */
    uint32_t t;
    uint32_t pad;
} rec_t;

static int rec_cmp(const void *x, const void *y)
{
    const rec_t *a = (const rec_t *)x, *b = (const rec_t *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->t != b->t) return a->t < b->t ? -1 : 1;
    return 0;
}

/* Returns the number m of unique undirected edges written to (u, v, t) with
 * u < v, or -1 if an endpoint is >= n, or -2 on allocation failure.  Output
 * arrays must hold n_edges entries.  ts may be NULL (all times 0).  out_dir,
 * if not NULL, receives per pair the directions its raw copies take: bit 0
 * for u -> v, bit 1 for v -> u. */
int64_t oracle_clean(uint32_t n, uint64_t n_edges, const uint32_t *src, const uint32_t *dst,
                     const uint32_t *ts, uint32_t *out_u, uint32_t *out_v, uint32_t *out_t, uint8_t *out_dir)
{
    rec_t *r = (rec_t *)malloc((n_edges ? n_edges : 1) * sizeof(rec_t));
    if (!r) return -2;
    uint64_t k = 0;
    for (uint64_t i = 0; i < n_edges; ++i) {
        const uint32_t a = src[i], b = dst[i];
        if (a >= n || b >= n) { free(r); return -1; }
        if (a == b) continue;
        const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        r[k].key = ((uint64_t)lo << 32) | hi;
        r[k].t = ts ? ts[i] : 0u;
        r[k].pad = a < b ? 1u : 2u;
        ++k;
    }
    qsort(r, k, sizeof(rec_t), rec_cmp);
    int64_t m = 0;
    for (uint64_t i = 0; i < k; ++i) {
        if (i > 0 && r[i].key == r[i - 1].key) {
            /* later copies are not earlier, but add their direction */
            if (out_dir) out_dir[m - 1] |= (uint8_t)r[i].pad;
            continue;
        }
        out_u[m] = (uint32_t)(r[i].key >> 32);
        out_v[m] = (uint32_t)(r[i].key & 0xffffffffu);
        out_t[m] = r[i].t;
        if (out_dir) out_dir[m] = (uint8_t)r[i].pad;
        ++m;
    }
    free(r);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Oriented graph: out-lists sorted by original id                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t n;
    uint64_t *start;   /* [n+1] */
    uint32_t *nbr;     /* [m] */
    uint32_t *tim;     /* [m] */
    uint64_t *deg;     /* [n] undirected degree d(v) of the cleaned graph */
    uint64_t *eid;     /* [m] position of each oriented edge in the cleaned list */
} orc_graph;

typedef struct {
    uint32_t v, t;
    uint64_t e;
} nb_t;

static int nb_cmp(const void *x, const void *y)
{
    const nb_t *a = (const nb_t *)x, *b = (const nb_t *)y;
    return a->v < b->v ? -1 : (a->v > b->v ? 1 : 0);
}

/* u comes before v in the degree order (ties broken by original id). */
static int before(const uint64_t *deg, uint32_t u, uint32_t v)
{
    if (deg[u] != deg[v]) return deg[u] < deg[v];
    return u < v;
}

static int orient(uint32_t n, uint64_t m, const uint32_t *eu, const uint32_t *ev, const uint32_t *et,
                  orc_graph *g)
{
    uint64_t *deg = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->n = n;
    g->start = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->nbr = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    g->tim = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    g->eid = (uint64_t *)malloc((m ? m : 1) * sizeof(uint64_t));
    uint64_t *fill = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    nb_t *tmp = NULL;
    if (!deg || !g->start || !g->nbr || !g->tim || !g->eid || !fill) goto oom;
    for (uint64_t i = 0; i < m; ++i) { deg[eu[i]]++; deg[ev[i]]++; }
    /* out-degree counts, then row starts */
    for (uint64_t i = 0; i < m; ++i) {
        const uint32_t s = before(deg, eu[i], ev[i]) ? eu[i] : ev[i];
        g->start[s + 1]++;
    }
    for (uint32_t v = 0; v < n; ++v) g->start[v + 1] += g->start[v];
    for (uint64_t i = 0; i < m; ++i) {
        const int fwd = before(deg, eu[i], ev[i]);
        const uint32_t s = fwd ? eu[i] : ev[i], d = fwd ? ev[i] : eu[i];
        const uint64_t at = g->start[s] + fill[s]++;
        g->nbr[at] = d;
        g->tim[at] = et[i];
        g->eid[at] = i;
    }
    /* sort each out-list by original id */
    uint64_t maxrow = 0;
    for (uint32_t v = 0; v < n; ++v) {
        const uint64_t len = g->start[v + 1] - g->start[v];
        if (len > maxrow) maxrow = len;
    }
    tmp = (nb_t *)malloc((maxrow ? maxrow : 1) * sizeof(nb_t));
    if (!tmp) goto oom;
    for (uint32_t v = 0; v < n; ++v) {
        const uint64_t b = g->start[v], len = g->start[v + 1] - b;
        for (uint64_t j = 0; j < len; ++j) {
            tmp[j].v = g->nbr[b + j];
            tmp[j].t = g->tim[b + j];
            tmp[j].e = g->eid[b + j];
        }
        qsort(tmp, len, sizeof(nb_t), nb_cmp);
        for (uint64_t j = 0; j < len; ++j) {
            g->nbr[b + j] = tmp[j].v;
            g->tim[b + j] = tmp[j].t;
            g->eid[b + j] = tmp[j].e;
        }
    }
    free(tmp);
    free(fill);
    g->deg = deg;
    return 0;
oom:
    free(tmp); free(fill); free(deg);
    free(g->start); free(g->nbr); free(g->tim); free(g->eid);
    g->start = NULL; g->nbr = NULL; g->tim = NULL; g->deg = NULL; g->eid = NULL;
    return -2;
}

static void free_graph(orc_graph *g)
{
    free(g->start); free(g->nbr); free(g->tim); free(g->deg); free(g->eid);
}

/* ------------------------------------------------------------------------ */
/* Survey (Algorithm 1 with the callbacks of Algorithms 2 and 4)             */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t a, b, c;          /* original ids, a < b < c */
    uint32_t t_ab, t_ac, t_bc; /* edge times */
    uint8_t l_a, l_b, l_c, pad;
} orc_tri;

static void emit_record(orc_tri *rec, uint32_t p, uint32_t q, uint32_t r,
                        uint32_t t_pq, uint32_t t_pr, uint32_t t_qr, const uint8_t *lab)
{
    /* put the three vertices in id order and carry each edge's time along */
    uint32_t v[3] = {p, q, r};
    uint32_t i, j;
    for (i = 0; i < 3; ++i)
        for (j = i + 1; j < 3; ++j)
            if (v[j] < v[i]) { uint32_t x = v[i]; v[i] = v[j]; v[j] = x; }
#define EDGE_T(x, y) ((((x) == p && (y) == q) || ((x) == q && (y) == p)) ? t_pq : \
                      ((((x) == p && (y) == r) || ((x) == r && (y) == p)) ? t_pr : t_qr))
    rec->a = v[0]; rec->b = v[1]; rec->c = v[2];
    rec->t_ab = EDGE_T(v[0], v[1]);
    rec->t_ac = EDGE_T(v[0], v[2]);
    rec->t_bc = EDGE_T(v[1], v[2]);
#undef EDGE_T
    rec->l_a = lab ? lab[v[0]] : 0;
    rec->l_b = lab ? lab[v[1]] : 0;
    rec->l_c = lab ? lab[v[2]] : 0;
    rec->pad = 0;
}

/*
 * Survey of the cleaned graph (u[i] < v[i], each pair once, times t[i]).
 * The Algorithm 3 output needs max_edge_shift < 32.
 * If `records` is non-NULL the triangles are also written there (at most
 * `capacity`; the count is returned in *n_records), in no particular order.
 * Returns 0, or -2 on allocation failure, -3 if a label >= n_labels is met
 * while the label table or mask is used.
 */
static int survey_impl(uint32_t n, uint64_t m, const uint32_t *eu, const uint32_t *ev, const uint32_t *et,
                       const uint8_t *edir, const uint8_t *vlab, const orc_spec *sp, orc_result *out, int n_threads,
                       orc_tri *records, uint64_t capacity, uint64_t *n_records,
                       uint32_t *maxe, uint64_t maxe_cap, uint64_t *n_maxe);

int oracle_survey(uint32_t n, uint64_t m, const uint32_t *eu, const uint32_t *ev, const uint32_t *et,
                  const uint8_t *edir, const uint8_t *vlab, const orc_spec *sp, orc_result *out, int n_threads,
                  orc_tri *records, uint64_t capacity, uint64_t *n_records)
{
    return survey_impl(n, m, eu, ev, et, edir, vlab, sp, out, n_threads, records, capacity, n_records, NULL, 0,
                       NULL);
}

/*
 * Algorithm 3's counting set, as its raw material (Section 4.5): for every
 * triangle of the cleaned graph whose three vertex labels are pairwise
 * distinct and that passes the spec's filters, the largest of its three
 * edge times, written to values[] (at most `capacity`, in no particular
 * order; their number in *n_values).  Counting equal values gives the set.
 * Returns as oracle_survey (the spec's outputs are surveyed too).
 */
int oracle_max_edge_values(uint32_t n, uint64_t m, const uint32_t *eu, const uint32_t *ev, const uint32_t *et,
                           const uint8_t *vlab, const orc_spec *sp, orc_result *out, int n_threads,
                           uint32_t *values, uint64_t capacity, uint64_t *n_values)
{
    return survey_impl(n, m, eu, ev, et, NULL, vlab, sp, out, n_threads, NULL, 0, NULL, values, capacity, n_values);
}

static int survey_impl(uint32_t n, uint64_t m, const uint32_t *eu, const uint32_t *ev, const uint32_t *et,
                       const uint8_t *edir, const uint8_t *vlab, const orc_spec *sp, orc_result *out, int n_threads,
                       orc_tri *records, uint64_t capacity, uint64_t *n_records,
                       uint32_t *maxe, uint64_t maxe_cap, uint64_t *n_maxe)
{
    orc_graph g;
    memset(out, 0, sizeof(*out));
    if ((sp->outputs & ORC_OUT_MAX_EDGE) && sp->max_edge_shift > 31) return -4;
    if ((sp->outputs & ORC_OUT_DIRECTED) && !edir) return -5;
    if ((sp->outputs & ORC_OUT_LABEL_TABLE || sp->filters & ORC_FILT_LABEL_MASK) && vlab) {
        for (uint32_t v = 0; v < n; ++v)
            if (vlab[v] >= sp->n_labels) return -3;
    }
    if (orient(n, m, eu, ev, et, &g) != 0) return -2;

    for (uint32_t p = 0; p < n; ++p) {
        const uint64_t d = g.start[p + 1] - g.start[p];
        out->wedges += d ? d * (d - 1) / 2 : 0;
    }

    uint64_t n_rec = 0, n_max = 0;
    int err = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        orc_result *acc = (orc_result *)calloc(1, sizeof(orc_result));
        if (!acc) {
#pragma omp atomic write
            err = -2;
        }
        int64_t p;
#pragma omp for schedule(dynamic, 64)
        for (p = 0; p < (int64_t)n; ++p) {
            if (!acc) continue;
            const uint64_t pb = g.start[p], pe = g.start[p + 1];
            for (uint64_t i = pb; i < pe; ++i) {
                const uint32_t q = g.nbr[i];
                const uint32_t t_pq = g.tim[i];
                /* merge Adj+(p) with Adj+(q), both sorted by id */
                uint64_t x = pb, y = g.start[q];
                const uint64_t ye = g.start[q + 1];
                while (x < pe && y < ye) {
                    if (g.nbr[x] < g.nbr[y]) { ++x; continue; }
                    if (g.nbr[x] > g.nbr[y]) { ++y; continue; }
                    const uint32_t r = g.nbr[x];
                    const uint32_t t_pr = g.tim[x], t_qr = g.tim[y];
                    const uint8_t l_p = vlab ? vlab[p] : 0, l_q = vlab ? vlab[q] : 0,
                                  l_r = vlab ? vlab[r] : 0;
                    uint32_t type = 0;
                    if (edir) {
                        const uint32_t P = (uint32_t)p;
                        type = oracle_directed_type(dir_from(P, q, edir[g.eid[i]]), dir_from(P, r, edir[g.eid[x]]),
                                                    dir_from(q, r, edir[g.eid[y]]));
                    }
                    callback(sp, acc, t_pq, t_pr, t_qr, l_p, l_q, l_r, g.deg[p], g.deg[q], g.deg[r], type);
                    if (records) {
                        uint64_t slot;
#pragma omp atomic capture
                        slot = n_rec++;
                        if (slot < capacity)
                            emit_record(&records[slot], (uint32_t)p, q, r, t_pq, t_pr, t_qr, vlab);
                    }
                    if (maxe && l_p != l_q && l_q != l_r && l_p != l_r &&
                        passes(sp, t_pq, t_pr, t_qr, l_p, l_q, l_r)) {
                        uint32_t t3 = t_pq > t_pr ? t_pq : t_pr;
                        if (t_qr > t3) t3 = t_qr;
                        uint64_t slot;
#pragma omp atomic capture
                        slot = n_max++;
                        if (slot < maxe_cap) maxe[slot] = t3;
                    }
                    ++x;
                    ++y;
                }
            }
        }
#pragma omp critical
        {
            if (acc) {
                out->triangles += acc->triangles;
                out->spread_count += acc->spread_count;
                for (int b = 0; b < 32; ++b) out->close_hist[b] += acc->close_hist[b];
                for (int b = 0; b < ORC_TABLE_MAX; ++b) out->label_table[b] += acc->label_table[b];
                for (int b = 0; b < 32 * 32; ++b) out->open_close[b] += acc->open_close[b];
                for (int b = 0; b < ORC_MAX_EDGE_BINS; ++b) out->max_edge[b] += acc->max_edge[b];
                for (int b = 0; b < ORC_DEGREE_MAX; ++b) out->degree_table[b] += acc->degree_table[b];
                for (int b = 0; b < 7; ++b) out->directed[b] += acc->directed[b];
            }
        }
        free(acc);
    }
    if (n_records) *n_records = n_rec;
    if (n_maxe) *n_maxe = n_max;
    free_graph(&g);
    return err;
}

/*
 * Local participation counts of the cleaned graph (u[i] < v[i], each pair
 * once): for every triangle that passes the spec's prefilters, one for each
 * of its three vertices (vcount, by original id, n entries) and each of its
 * three edges (ecount, by position in the cleaned list, m entries).  Either
 * output may be NULL.  Returns 0, -2 on allocation failure, -3 for a label
 * >= n_labels while the label mask is used.
 */
int oracle_participation(uint32_t n, uint64_t m, const uint32_t *eu, const uint32_t *ev, const uint32_t *et,
                         const uint8_t *vlab, const orc_spec *sp, uint64_t *vcount, uint64_t *ecount,
                         int n_threads)
{
    orc_graph g;
    if (vcount) memset(vcount, 0, (size_t)n * sizeof(uint64_t));
    if (ecount) memset(ecount, 0, (size_t)m * sizeof(uint64_t));
    if ((sp->filters & ORC_FILT_LABEL_MASK) && vlab) {
        for (uint32_t v = 0; v < n; ++v)
            if (vlab[v] >= sp->n_labels) return -3;
    }
    if (orient(n, m, eu, ev, et, &g) != 0) return -2;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int64_t p;
#pragma omp parallel for schedule(dynamic, 64)
    for (p = 0; p < (int64_t)n; ++p) {
        const uint64_t pb = g.start[p], pe = g.start[p + 1];
        for (uint64_t i = pb; i < pe; ++i) {
            const uint32_t q = g.nbr[i];
            uint64_t x = pb, y = g.start[q];
            const uint64_t ye = g.start[q + 1];
            while (x < pe && y < ye) {
                if (g.nbr[x] < g.nbr[y]) { ++x; continue; }
                if (g.nbr[x] > g.nbr[y]) { ++y; continue; }
                const uint32_t r = g.nbr[x];
                const uint8_t l_p = vlab ? vlab[p] : 0, l_q = vlab ? vlab[q] : 0, l_r = vlab ? vlab[r] : 0;
                if (passes(sp, g.tim[i], g.tim[x], g.tim[y], l_p, l_q, l_r)) {
                    if (vcount) {
#pragma omp atomic
                        vcount[p] += 1;
#pragma omp atomic
                        vcount[q] += 1;
#pragma omp atomic
                        vcount[r] += 1;
                    }
                    if (ecount) {
#pragma omp atomic
                        ecount[g.eid[i]] += 1;
#pragma omp atomic
                        ecount[g.eid[x]] += 1;
#pragma omp atomic
                        ecount[g.eid[y]] += 1;
                    }
                }
                ++x;
                ++y;
            }
        }
    }
    free_graph(&g);
    return 0;
}

/* Sizes of the structs, so a binding can check its own layout. */
uint64_t oracle_sizeof_spec(void) { return sizeof(orc_spec); }
uint64_t oracle_sizeof_result(void) { return sizeof(orc_result); }
uint64_t oracle_sizeof_tri(void) { return sizeof(orc_tri); }
