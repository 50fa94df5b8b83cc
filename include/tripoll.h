/*
 * tripoll.h -- C ABI of the MI355X (gfx950) metadata triangle survey.
 *
 * The operation is the triangle survey of Steil et al., "TriPoll: Computing
 * Surveys of Triangles in Massive-Scale Temporal Graphs with Metadata":
 * every triangle of an undirected graph decorated with vertex and edge
 * metadata is found exactly once on the degree-ordered directed graph
 * (Preliminaries; Graph Storage subsection), and the six metadata items of
 * each triangle are handed to a callback that reduces them into counters
 * (Algorithm 1; Callback Examples subsection).  The arbitrary callback of the
 * paper is replaced here by a closed menu of reductions (TP_OUT_*) and
 * prefilters (TP_FILT_*); results are the counters' final values.
 *
 * Metadata carried: one uint32 time per edge and one uint8 label per vertex.
 *
 * Conventions for every entry point:
 *   - The return value is a tp_status; nothing aborts or throws across the
 *     ABI.  On a non-OK status, tripoll_last_error() returns a message for
 *     the calling thread and the caller's output arguments are untouched.
 *   - Input arrays are borrowed for the duration of the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is ordered on that stream; calls documented as synchronous return
 *     only after their work has completed.
 *   - Objects returned through `**out` are owned by the caller and released
 *     with the matching *_free call.  A graph is immutable after it is built
 *     and may be surveyed concurrently from several streams.
 *   - All counters are uint64 and exact.
 */
#ifndef TRIPOLL_H
#define TRIPOLL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TP_OK = 0,
    TP_ERR_INVALID = 1,     /* bad argument or input (id >= n, label >= n_labels, ...) */
    TP_ERR_OOM = 2,         /* device or host allocation failed; nothing leaked */
    TP_ERR_DEVICE = 3,      /* a HIP call failed */
    TP_ERR_BUSY = 4,        /* server queue or slot table full */
    TP_ERR_UNSUPPORTED = 5, /* valid but not supported (e.g. no gfx950 device) */
    TP_ERR_NOT_FOUND = 6    /* unknown handle or ticket */
} tp_status;

/* Where the arrays of a tp_edge_list live. */
#define TP_MEM_HOST 0u
#define TP_MEM_DEVICE 1u

/* Tie-break `hash` of the degree order (Preliminaries): vertices of equal
 * degree are ordered by hash(v).  Survey results do not depend on it. */
#define TP_TIE_MIX 0u /* a bijective integer mix of the vertex id (default) */
#define TP_TIE_ID 1u  /* the vertex id itself */

/*
 * A raw undirected edge list (Preliminaries: the input graph is undirected;
 * Datasets subsection: a multigraph keeps the chronologically first edge).
 * Edges may repeat, in either direction; self-loops are allowed and ignored.
 * Each unordered pair {u,v} becomes one edge whose time is the minimum over
 * all of its copies.
 *   n_vertices    ids are in [0, n_vertices); n_vertices < 2^32 - 1
 *   n_edges       number of raw edges (uint64)
 *   src, dst      uint32[n_edges]
 *   edge_time     uint32[n_edges], or NULL: every time is 0 (the paper's
 *                 dummy metadata for plain counting, Triangle Counting
 *                 subsection of the evaluation)
 *   vertex_label  uint8[n_vertices], or NULL: every label is 0
 *   mem_space     TP_MEM_HOST or TP_MEM_DEVICE, for all four arrays
 *   tie_hash      TP_TIE_MIX or TP_TIE_ID
 *   flags         0, or TP_EDGES_DIRECTED: edges are arcs src -> dst.  The
 *                 graph is still surveyed as undirected, but each oriented
 *                 edge keeps two bits of the directions its copies take (the
 *                 remark on directed inputs at the end of the Preliminaries'
 *                 storage discussion), for the DIRECTED census; needs
 *                 n_vertices <= 2^31
 */
#define TP_EDGES_DIRECTED 0x1u
typedef struct {
    uint32_t n_vertices;
    uint32_t mem_space;
    uint64_t n_edges;
    const uint32_t *src;
    const uint32_t *dst;
    const uint32_t *edge_time;
    const uint8_t *vertex_label;
    uint32_t tie_hash;
    uint32_t flags;
} tp_edge_list;

typedef struct tp_graph tp_graph;

/* Target classes of the survey plan, by d+(q) (the out-degree of the middle
 * vertex of a wedge): 0 tiny d+ <= 51, 1 small <= 819, 2 large <= 3276,
 * 3 huge.  The class decides where Adj+(q) is kept while the wedges through
 * q are checked.  A huge target's Adj+(q) is cut into ceil(d+ / 3276) runs
 * of consecutive ranks (pieces), each checked against only the candidates
 * in its rank range; the planner cuts the in-edge records accordingly. */
#define TP_NUM_CLASSES 4

/* Graph statistics.  Degrees are of the cleaned simple graph; d+ is the
 * out-degree in the degree-ordered directed graph; wedges = |W+| = sum over
 * v of C(d+(v), 2), the wedge checks of the survey (Preliminaries). */
typedef struct {
    uint64_t n_vertices;
    uint64_t n_raw_edges;
    uint64_t n_self_loops;
    uint64_t n_edges;          /* unique undirected edges m */
    uint64_t d_max;
    uint64_t dplus_max;
    uint64_t wedges;           /* |W+| */
    uint64_t probes;           /* wedge checks the survey issues (|W+| minus wedges whose
                                  middle vertex has no out-edge, which cannot close) */
    uint64_t n_targets;        /* vertices q with at least one wedge to check */
    uint64_t n_tiles;          /* work tiles of the survey plan */
    uint64_t device_bytes;     /* HBM held by the graph */
    uint32_t max_label;
    uint32_t reserved;
    float phase_ms[8];         /* device time of the build phases: 0 validate+canonicalise,
                                  1 sort by pair, 2 dedup, 3 degree+order, 4 orient+sort,
                                  5 CSR+metadata, 6 in-edge index, 7 survey plan */
    float build_ms;            /* sum of phase_ms */
    uint32_t reserved2;
    /* survey plan per target class (TP_NUM_CLASSES) */
    uint64_t class_tiles[TP_NUM_CLASSES];   /* tiles */
    uint64_t class_records[TP_NUM_CLASSES]; /* in-edge records (one per oriented edge p -> q) */
    uint64_t class_staged[TP_NUM_CLASSES];  /* sum over tiles of d+(q): out-list entries loaded
                                               per survey */
    uint64_t class_probes[TP_NUM_CLASSES];  /* wedge checks */
} tp_graph_stats;

/*
 * Build the degree-ordered directed graph with co-located metadata
 * (Preliminaries; Graph Storage subsection, Adj+^m(u) with meta(u,v) and
 * meta(v) stored beside each out-neighbour v).  Synchronous.
 *   edges   the raw edge list (see tp_edge_list); borrowed
 *   stream  hipStream_t as void*
 *   out     receives a new graph on TP_OK
 * Errors: TP_ERR_INVALID for NULL pointers with n_edges > 0, an id >= n, or
 * n_vertices >= 2^32 - 1; TP_ERR_OOM; TP_ERR_DEVICE.
 */
tp_status tripoll_build(const tp_edge_list *edges, void *stream, tp_graph **out);

/* Statistics of a built graph (host struct, filled synchronously). */
tp_status tripoll_graph_stats(const tp_graph *g, tp_graph_stats *out);

/* Release a graph and its device memory.  NULL is accepted. */
tp_status tripoll_graph_free(tp_graph *g);

/*
 * Copy the oriented graph to host arrays, for inspection and tests.  Any
 * pointer may be NULL to skip that array.  Vertices are numbered by their
 * position in the degree order (rank); row v of the CSR lists the
 * out-neighbours of rank v in increasing rank.
 *   rowptr   uint64[n+1]    col  uint32[m]  (ranks)
 *   etime    uint32[m]      time of each oriented edge
 *   tlabel   uint8[m]       label of each edge's target
 *   rank_to_id uint32[n]    original id of each rank
 *   rank_label uint8[n]     label of each rank
 */
tp_status tripoll_graph_export(const tp_graph *g, uint64_t *rowptr, uint32_t *col, uint32_t *etime,
                               uint8_t *tlabel, uint32_t *rank_to_id, uint8_t *rank_label);

/* ------------------------------------------------------------------------ */
/* Survey                                                                    */
/* ------------------------------------------------------------------------ */

/* Reductions (the callback of Algorithm 1), selected as a bitmask.  For each
 * triangle with edge times t1 <= t2 <= t3 and vertex labels a <= b <= c:
 *   COUNT        triangles += 1                         (Algorithm 2)
 *   CLOSE_HIST   close_hist[bin(t3 - t1)] += 1           (Algorithm 4, closing time)
 *   LABEL_TABLE  label_table[C(c+2,3)+C(b+1,2)+a] += 1   (label-multiset survey)
 *   SPREAD_COUNT spread_count += (t3 - t1 < spread_lt)
 *   OPEN_CLOSE   open_close[32*bin(t2 - t1) + bin(t3 - t1)] += 1 (Algorithm 4, joint)
 *   MAX_EDGE     if a, b, c are pairwise distinct:
 *                max_edge[min(1023, t3 >> max_edge_shift)] += 1
 *                (Algorithm 3: the distribution of the largest edge metadata
 *                over triangles whose vertex labels all differ; the paper's
 *                counting set of exact values is kept per 2^max_edge_shift
 *                range of t3, exact when every t3 >> shift < 1024)
 *   DIRECTED     directed[type] += 1 on a graph built with TP_EDGES_DIRECTED,
 *                type of the triangle's arcs as in the triad census:
 *                0 030T (three one-way arcs, no cycle), 1 030C (a 3-cycle),
 *                2 120D, 3 120U, 4 120C (one mutual pair; the third vertex
 *                sends both its arcs, receives both, or one of each),
 *                5 210 (two mutual pairs), 6 300 (three mutual pairs)
 *   DEGREE_TABLE with x <= y <= z the values bin(d(v)) of the three vertices
 *                (d the undirected degree of the cleaned graph):
 *                degree_table[C(z+2,3)+C(y+1,2)+x] += 1
 *                (the degree-metadata survey of the evaluation, which counts
 *                triples of ceil(log2 d) of p, q, r; in the degree order
 *                d(p) <= d(q) <= d(r), so that triple is already sorted)
 * with bin(D) = 0 for D <= 1 and min(31, ceil(log2 D)) otherwise, computed
 * exactly in integers.  The triangle count is always produced.  Every
 * output is produced by the single-graph surveys, by batch surveys (per
 * graph) and by served requests; tripoll_survey on a batch handle (the
 * union's totals) does not produce DEGREE_TABLE. */
#define TP_OUT_COUNT 0x01u
#define TP_OUT_CLOSE_HIST 0x02u
#define TP_OUT_LABEL_TABLE 0x04u
#define TP_OUT_SPREAD_COUNT 0x08u
#define TP_OUT_OPEN_CLOSE 0x10u
#define TP_OUT_MAX_EDGE 0x20u
#define TP_OUT_DEGREE_TABLE 0x40u
#define TP_OUT_DIRECTED 0x80u

/* Prefilters applied before every reduction (the conditional of the
 * callbacks in Algorithms 3 and 4):
 *   WINDOW      keep triangles whose three edge times all lie in [t_lo, t_hi]
 *   LABEL_MASK  keep triangles whose label-multiset index has its bit set */
#define TP_FILT_WINDOW 0x01u
#define TP_FILT_LABEL_MASK 0x02u

#define TP_MAX_LABELS 16u
#define TP_TABLE_MAX 816u /* C(16+2, 3) */
#define TP_MAX_EDGE_BINS 1024u
#define TP_DEGREE_MAX 5984u /* C(32+2, 3): three values in 0..31 */

/* Intersection strategy (tests and tuning).  AUTO picks per target vertex. */
#define TP_STRAT_AUTO 0u
#define TP_STRAT_GLOBAL_SEARCH 1u /* binary search of Adj+(q) in HBM for every target */
#define TP_STRAT_TABLE_STRESS 2u  /* LDS tables with one placement attempt per key: exercises
                                     the stash and the HBM fallback (slow; for tests) */

/* How a target class searches Adj+(q) (survey plan variants):
 *   TP_VAR_DEFAULT      the class's own choice: per-wave LDS tables (tiny),
 *                       per-workgroup LDS tables (small, large, and huge
 *                       one piece at a time)
 *   TP_VAR_WAVE_TABLE   LDS cuckoo tables, one per wave (tiny class only)
 *   TP_VAR_GROUP_TABLE  LDS cuckoo tables, one per workgroup
 *   TP_VAR_SEARCH       binary search of Adj+(q) in HBM, a workgroup per tile
 *   TP_VAR_WAVE_SEARCH  binary search of Adj+(q) in HBM, a wave per tile */
#define TP_VAR_DEFAULT 0u
#define TP_VAR_WAVE_TABLE 1u
#define TP_VAR_GROUP_TABLE 2u
#define TP_VAR_SEARCH 3u
#define TP_VAR_WAVE_SEARCH 4u

typedef struct {
    uint32_t outputs;        /* TP_OUT_* bitmask */
    uint32_t filters;        /* TP_FILT_* bitmask */
    uint32_t n_labels;       /* L in 1..16, labels must be < L when LABEL_TABLE or
                                LABEL_MASK is used; the table has C(L+2,3) entries */
    uint32_t strategy;       /* TP_STRAT_* */
    uint64_t spread_lt;      /* SPREAD_COUNT threshold */
    uint64_t t_lo, t_hi;     /* WINDOW bounds, closed; t_lo <= t_hi */
    uint64_t label_mask[13]; /* LABEL_MASK bitset over multiset indices */
    uint32_t max_edge_shift; /* MAX_EDGE bin width 2^max_edge_shift, 0..31 */
    uint32_t reserved;       /* must be 0 */
} tp_survey_spec;

/* Host result.  Unrequested outputs are zero. */
typedef struct {
    uint64_t triangles;      /* triangles passing the filters */
    uint64_t spread_count;
    uint64_t probes;         /* wedge checks performed */
    uint64_t close_hist[32];
    uint64_t label_table[TP_TABLE_MAX];
    uint64_t open_close[32 * 32];
    uint64_t max_edge[TP_MAX_EDGE_BINS];
    uint64_t degree_table[TP_DEGREE_MAX];
    uint64_t directed[8];    /* the seven types of DIRECTED, then 0 */
    float kernel_ms;         /* device time of the intersection kernels */
    float total_ms;          /* device time of the whole survey call */
    float class_ms[TP_NUM_CLASSES]; /* device time of the kernel of each target class */
    uint64_t class_triangles[TP_NUM_CLASSES]; /* triangles counted by each target class's kernel
                                                 (their sum is `triangles`) */
} tp_survey_result;

/* Word layout of a device result buffer (uint64[TP_RESULT_WORDS]).  The
 * last TP_RW_SCRATCH_WORDS words are used by the survey itself: the first
 * four are work counters whose content is unspecified; then, at
 * TP_RW_CLASS_TRI + c, the triangles counted by target classes 0..c (a
 * running sum, taken after each class's kernel); the last eight are work
 * counters again. */
#define TP_RW_TRIANGLES 0u
#define TP_RW_SPREAD 1u
#define TP_RW_PROBES 2u
#define TP_RW_HIST 3u
#define TP_RW_TABLE (TP_RW_HIST + 32u)
#define TP_RW_OPEN_CLOSE (TP_RW_TABLE + TP_TABLE_MAX)
#define TP_RW_MAX_EDGE (TP_RW_OPEN_CLOSE + 1024u)
#define TP_RW_DEGREE (TP_RW_MAX_EDGE + TP_MAX_EDGE_BINS)
#define TP_RW_DIRECTED (TP_RW_DEGREE + TP_DEGREE_MAX)
#define TP_RW_SCRATCH (TP_RW_DIRECTED + 8u)
#define TP_RW_SCRATCH_WORDS 16u
#define TP_RW_CLASS_TRI (TP_RW_SCRATCH + 4u)
#define TP_RESULT_WORDS (TP_RW_SCRATCH + TP_RW_SCRATCH_WORDS)

/*
 * Survey a graph (Algorithm 1 with the reductions above).  Synchronous: the
 * result is on the host when it returns.
 * Errors: TP_ERR_INVALID for NULL arguments, n_labels outside 1..16, a graph
 * label >= n_labels when labels are used, t_lo > t_hi, max_edge_shift > 31,
 * reserved != 0, or DIRECTED on a graph built without TP_EDGES_DIRECTED;
 * TP_ERR_UNSUPPORTED for DEGREE_TABLE on a batch handle (use
 * tripoll_survey_batch);
 * TP_ERR_DEVICE.
 */
tp_status tripoll_survey(const tp_graph *g, const tp_survey_spec *spec, tp_survey_result *out,
                         void *stream);

/*
 * As tripoll_survey, but enqueued on `stream` without waiting and without
 * allocating.  `dev_out` is a device buffer of TP_RESULT_WORDS uint64 owned by
 * the caller; it is overwritten (zeroed, then accumulated) by work ordered on
 * `stream`, and must not be shared by surveys in flight at the same time.
 */
tp_status tripoll_survey_async(const tp_graph *g, const tp_survey_spec *spec, uint64_t *dev_out,
                               void *stream);

/*
 * The exact counting set of Algorithm 3 (Section 4.5, "Containers" in
 * Section 4.1): over the triangles whose three vertex labels are pairwise
 * distinct and that pass the spec's filters, every distinct value of the
 * largest of the three edge times, with the number of triangles that have
 * it.  (TP_OUT_MAX_EDGE reports the same triangles binned into 1024 ranges
 * of 2^max_edge_shift times; this call keeps every value.)
 *   spec        filters, n_labels and strategy apply as in tripoll_survey;
 *               outputs and max_edge_shift are ignored
 *   dev_values  device buffer of `capacity` uint32 owned by the caller: the
 *               distinct largest times, ascending
 *   dev_counts  device buffer of `capacity` uint64 owned by the caller: the
 *               number of triangles of each value
 *   n_values    host: the number of distinct values written
 * Synchronous with respect to the host.  Works in a device table of 2^k >=
 * 2 m entries of 16 bytes (m: oriented edges, at most 2^32 entries),
 * allocated for the call; each counted triangle costs two device-scope
 * atomics there, so the call is slower than the binned output.  At most m
 * values exist, so capacity = m always suffices.
 * Errors: TP_ERR_INVALID for a null pointer or a spec tripoll_survey
 * refuses, and when more than `capacity` distinct values exist (then
 * *n_values holds their number and the buffers are untouched);
 * TP_ERR_UNSUPPORTED on a batch handle; TP_ERR_OOM; TP_ERR_DEVICE.
 */
tp_status tripoll_max_edge_counts(const tp_graph *g, const tp_survey_spec *spec, uint32_t *dev_values,
                                  uint64_t *dev_counts, uint64_t capacity, uint64_t *n_values, void *stream);

/*
 * As tripoll_survey, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the survey's device result words and work counters live in a
 * static device array of TP_RESULT_WORDS uint64 (about 71 KB) that each GPU
 * holds from the first call on it until the process ends, so the call makes
 * no device allocation and releases nothing.  The result size does not
 * depend on the graph or the spec, so every survey fits that array.
 * Synchronous; kernel_ms, total_ms and class_ms are 0 (no timers).
 *   The graph's device must be the current device.
 *   All calls on one GPU share its array, which keeps the last call's
 *   contents (each call clears it first): calls that overlap on one GPU,
 *   from several threads or streams, race and must not be made.
 * Errors: as tripoll_survey; TP_ERR_INVALID also when the current device is
 * not the graph's.  On TP_ERR_DEVICE *out may have been partly written.
 */
tp_status tripoll_survey_noalloc(const tp_graph *g, const tp_survey_spec *spec, tp_survey_result *out,
                                 void *stream);

/*
 * Enumerate every triangle (the full-enumeration use of the callback,
 * Introduction).  Writes up to `capacity` records of 9 uint32 each into the
 * device buffer `dev_records`: original ids a, b, c (the triangle's pivot,
 * middle and top vertex in the degree order), the times of edges ab, ac, bc,
 * and the labels of a, b, c.  *n_found receives the number of triangles,
 * which may exceed capacity (then only `capacity` records were written).
 * Synchronous.
 */
tp_status tripoll_enumerate(const tp_graph *g, uint32_t *dev_records, uint64_t capacity,
                            uint64_t *n_found, void *stream);

/*
 * Streamed enumeration: every triangle exactly once, in chunks that never
 * overflow the caller's buffer (the full-enumeration use of the callback,
 * Introduction, with the caller draining the buffer between chunks).
 * tripoll_enum_open counts the triangles of every tile of the survey plan
 * (one pass), so that each tile's records have a known place; each
 * tripoll_enum_next then writes the records of as many whole tiles as fit
 * in `capacity`, in the record format of tripoll_enumerate, and sets
 * *n_written (0 once every record was written).  The spec's prefilters
 * apply; its outputs are ignored.  Calls on one stream object must not
 * overlap; the graph must outlive it.
 *   total     host; receives the number of records the stream will produce
 *   max_tile  host; receives the records of the largest tile: a capacity of
 *             at least this always makes progress
 * Errors: TP_ERR_INVALID for bad arguments, or when `capacity` is below the
 * next tile's records (nothing is written then); as tripoll_survey otherwise.
 */
typedef struct tp_enum_stream tp_enum_stream;
tp_status tripoll_enum_open(const tp_graph *g, const tp_survey_spec *spec, void *stream, tp_enum_stream **out,
                            uint64_t *total, uint64_t *max_tile);
tp_status tripoll_enum_next(tp_enum_stream *e, uint32_t *dev_records, uint64_t capacity, uint64_t *n_written,
                            void *stream);
tp_status tripoll_enum_close(tp_enum_stream *e);

/*
 * Local participation counts (Introduction; the Triangle Counting
 * subsection of the evaluation: the per-vertex counts behind clustering
 * coefficients and the per-edge counts behind truss decomposition).  For
 * every triangle that passes the spec's prefilters (WINDOW, LABEL_MASK; the
 * spec's outputs are ignored), one is added to the counter of each of its
 * three vertices and each of its three edges.  Synchronous.
 *   vertex_counts  device uint64[n_vertices] indexed by original vertex id,
 *                  overwritten; or NULL
 *   edge_counts    device uint64[n_edges] indexed by CSR slot of the oriented
 *                  graph (tripoll_graph_export gives each slot's endpoints:
 *                  row = rank of one end, col = rank of the other), overwritten;
 *                  or NULL (then a temporary is allocated)
 *   triangles      host; receives the number of triangles counted; or NULL
 * The sums of both arrays are three times *triangles.
 * On a batch handle the counts are those of the union of its graphs (no
 * triangle spans two graphs): vertex ids are the batch's global ids (graph
 * g's vertices follow those of graphs 0 .. g-1), the ranks and CSR slots of
 * graph g are contiguous and follow those of graphs 0 .. g-1, and
 * *triangles is the batch's total.
 * Errors: as tripoll_survey.
 */
tp_status tripoll_participation(const tp_graph *g, const tp_survey_spec *spec, uint64_t *vertex_counts,
                                uint64_t *edge_counts, uint64_t *triangles, void *stream);

/* ------------------------------------------------------------------------ */
/* Batches of independent graphs                                             */
/* ------------------------------------------------------------------------ */

/*
 * Many independent raw edge lists, built and surveyed together.  A batch is
 * one disjoint union; every graph is cleaned and degree-ordered within
 * itself (Preliminaries), and since no triangle spans two graphs the survey
 * of the union, split per graph, is the survey of each graph (Algorithm 1 on
 * each part).  Graph g owns raw edges [edge_offsets[g], edge_offsets[g+1])
 * of src/dst/edge_time, whose ids are local to it, in [0, vertex_counts[g]);
 * its labels are vertex_label[voff[g] + i] for local id i, where voff is the
 * running sum of vertex_counts (voff[0] = 0).
 *   n_graphs       >= 1
 *   edge_offsets   uint64[n_graphs + 1] in host memory; edge_offsets[0] = 0,
 *                  non-decreasing; the last entry is the total raw edge count
 *   vertex_counts  uint32[n_graphs] in host memory; 0 allowed (a graph with
 *                  no vertices must own no edges); the sum is < 2^32 - 1
 *   src, dst, edge_time, vertex_label, mem_space, tie_hash: as in
 *                  tp_edge_list, concatenated over the graphs
 *   flags          0, or TP_EDGES_DIRECTED (every graph's edges are arcs
 *                  src -> dst, kept for the DIRECTED census as in tp_edge_list)
 */
typedef struct {
    uint32_t n_graphs;
    uint32_t mem_space;
    const uint64_t *edge_offsets;
    const uint32_t *vertex_counts;
    const uint32_t *src;
    const uint32_t *dst;
    const uint32_t *edge_time;
    const uint8_t *vertex_label;
    uint32_t tie_hash;
    uint32_t flags;
} tp_batch_edges;

/*
 * Build a batch as one tp_graph whose vertices are grouped by graph (graph
 * g holds ranks [voff[g], voff[g+1]) of the degree order).  The whole batch
 * shares one survey plan, so one persistent kernel per target class covers
 * every graph.  Synchronous.  Graph statistics are those of the union.
 * Errors: as tripoll_build; TP_ERR_INVALID also for decreasing offsets, an
 * edge whose local id is >= its graph's vertex count, or a batch whose
 * graph, degree and vertex bits exceed one 64-bit order key.
 */
tp_status tripoll_build_batch(const tp_batch_edges *batch, void *stream, tp_graph **out);

/* Number of graphs of a batch (1 for a graph from tripoll_build). */
tp_status tripoll_graph_count(const tp_graph *g, uint32_t *n_graphs);

/*
 * Per-graph result block of a batch survey, in uint64 words:
 *   [TP_BW_TRIANGLES] [TP_BW_SPREAD] [TP_BW_PROBES] [TP_BW_HIST, +32)
 *   then C(n_labels+2, 3) label-table words if LABEL_TABLE is requested,
 *   then 32*32 open/close words if OPEN_CLOSE is requested,
 *   then TP_MAX_EDGE_BINS max-edge words if MAX_EDGE is requested,
 *   then TP_DEGREE_MAX degree-table words if DEGREE_TABLE is requested
 *   (each graph's degrees are its own),
 *   then 8 directed-census words if DIRECTED is requested (the batch must be
 *   built with TP_EDGES_DIRECTED).
 * tripoll_batch_words(spec) returns the block length (0 for a NULL spec).
 */
#define TP_BW_TRIANGLES 0u
#define TP_BW_SPREAD 1u
#define TP_BW_PROBES 2u
#define TP_BW_HIST 3u
#define TP_BW_TABLE 35u
#define TP_BATCH_SCRATCH_WORDS 8u
uint64_t tripoll_batch_words(const tp_survey_spec *spec);

/*
 * Survey every graph of a batch (Algorithm 1 with the reductions above,
 * reported per graph).  Enqueued on `stream`; allocates nothing; may be
 * recorded into a HIP graph by the caller.
 *   dev_out  device buffer of n_graphs * tripoll_batch_words(spec) +
 *            TP_BATCH_SCRATCH_WORDS uint64, owned by the caller: block g
 *            starts at word g * tripoll_batch_words(spec); the last
 *            TP_BATCH_SCRATCH_WORDS words are work counters.  Overwritten
 *            by work ordered on `stream`; one survey in flight per buffer.
 * Errors: as tripoll_survey.
 */
tp_status tripoll_survey_batch(const tp_graph *g, const tp_survey_spec *spec, uint64_t *dev_out, void *stream);

/*
 * A recorded survey launch: the fills and persistent kernels of
 * tripoll_survey_batch for one graph, spec and output buffer, captured once
 * into an executable HIP graph and replayed with one launch call.
 *   tripoll_survey_capture  records it (synchronous); `dev_out` as for
 *                           tripoll_survey_batch and bound to the launch.
 *                           Recording runs one survey first, on a private
 *                           stream into a temporary buffer of its own (so
 *                           that every kernel is set up before the capture);
 *                           it does not write dev_out, which only replays do
 *   tripoll_launch_replay   enqueues one replay on `stream`; replays on one
 *                           launch must not overlap (they share dev_out)
 *   tripoll_launch_free     releases it (NULL accepted); the graph must
 *                           outlive the launch
 */
typedef struct tp_launch tp_launch;
tp_status tripoll_survey_capture(const tp_graph *g, const tp_survey_spec *spec, uint64_t *dev_out,
                                 tp_launch **out);
tp_status tripoll_launch_replay(tp_launch *launch, void *stream);
tp_status tripoll_launch_free(tp_launch *launch);

/* ------------------------------------------------------------------------ */
/* Survey plan and autotuning                                                */
/* ------------------------------------------------------------------------ */

/*
 * The survey plan of a graph: per target class, the search variant
 * (TP_VAR_*) and the cap on in-edge records per tile (a tile is the unit of
 * work one workgroup or wave claims; a target with more records, or more
 * than 256 wedge checks per record of cap, is cut into several interleaved
 * tiles).  Results never depend on the plan, only the time does.
 *   tile_records  power of two in [16, 65536]
 */
typedef struct {
    uint32_t variant[TP_NUM_CLASSES];
    uint32_t tile_records[TP_NUM_CLASSES];
} tp_plan;

/* Read the plan of a graph (host struct). */
tp_status tripoll_get_plan(const tp_graph *g, tp_plan *out);

/*
 * Replace the plan of a graph (re-cuts the tiles on `stream`; synchronous).
 * Not to be called while surveys of the graph are in flight.
 * Errors: TP_ERR_INVALID for an unknown variant, a variant the class cannot
 * use (per-wave tables outside the tiny class) or
 * a tile cap that is not a power of two in [16, 65536].
 */
tp_status tripoll_set_plan(tp_graph *g, const tp_plan *plan, void *stream);

/* Outcome of tripoll_tune. */
typedef struct {
    tp_plan chosen;                    /* the plan now set on the graph */
    float default_ms[TP_NUM_CLASSES];  /* kernel time of each class under the default plan */
    float tuned_ms[TP_NUM_CLASSES];    /* kernel time of each class under the chosen plan */
    uint32_t trials;                   /* timed (class, variant, tile cap) launches */
    uint32_t reserved;
} tp_tune_result;

/*
 * Autotune the plan for one survey kind: for every class, time each usable
 * variant at tile caps 256, 1024, 4096 and 16384 with the survey `spec` on
 * this graph, and keep the fastest per class (the default -- the class's own
 * variant, 1024 records per tile, 16384 for the large class -- stays unless
 * another beats it by more than 3%).  Runs real surveys (cost: a few times one
 * survey).  Synchronous; sets the plan on the graph.  Not to be called while
 * surveys of the graph are in flight.
 */
tp_status tripoll_tune(tp_graph *g, const tp_survey_spec *spec, void *stream, tp_tune_result *out);

/* ------------------------------------------------------------------------ */
/* Served mode                                                               */
/* ------------------------------------------------------------------------ */

/*
 * A survey server keeps graphs resident on the device and answers survey
 * requests against them as they arrive (Algorithm 1 with the reductions
 * above, one request per survey).  Requests on one graph share passes over
 * its work (continuous batching): the pass is cut into segments, every step
 * surveys one segment for all requests that hold one of the graph's slots,
 * and each triangle is reduced into the counters of each such request with
 * that request's own filters.  A request that arrives while a pass is on the
 * device takes a free slot at the next step and is complete once it has
 * seen every segment once (wrapping round the end of the pass); its result
 * equals that of tripoll_survey on the same graph and spec.  Graphs with
 * little work (one segment) run on a second stream and overlap the steps of
 * large ones.  Device memory -- resident graphs and per-request buffers --
 * is admitted against the server's budget.  A worker thread owned by the
 * server drives the device; all functions are thread-safe.
 *
 * Served survey kinds: every output and filter of tripoll_survey.  Requests
 * for COUNT, CLOSE_HIST, LABEL_TABLE and SPREAD_COUNT share each step's
 * pass; requests that also ask for OPEN_CLOSE, MAX_EDGE, DEGREE_TABLE or
 * DIRECTED (whose counters do not fit the shared pass's LDS) take part in
 * the same steps and segments but run the single-request kernels over each
 * segment into result words of their own (their memory is
 * TP_RESULT_WORDS * 8 bytes of the budget).
 */
typedef struct tp_server tp_server;

#define TP_SERVER_TAGS 8u /* latency statistics are kept per tag 0..7 */

typedef struct {
    uint32_t max_slots;   /* request slots per resident graph, 1..16 (0: 8) */
    uint32_t n_labels;    /* label range of every label output or filter, 1..16
                             (0: 8); graphs used with them need labels < n_labels */
    uint64_t hbm_budget;  /* device bytes the server may hold: resident graphs plus
                             request buffers (0: 90% of the free device memory) */
    uint64_t step_wedges; /* wedge checks per step, the admission granularity
                             (0: 2^34) */
    uint32_t max_queue;   /* waiting requests before submit says TP_ERR_BUSY (0: 4096) */
    uint32_t reserved;
} tp_server_config;

/* Per-request timing.  Times are microseconds on the server's clock. */
typedef struct {
    uint32_t tag;
    uint32_t steps;         /* steps the request took part in */
    double arrival_us;      /* tripoll_server_submit returned */
    double admit_us;        /* it took a slot */
    double done_us;         /* its result reached host memory */
} tp_request_info;

typedef struct {
    uint64_t submitted, completed, rejected;   /* rejected: submit said BUSY */
    uint64_t waiting, running;                 /* now */
    uint64_t steps;                            /* device steps issued */
    uint64_t triangles;                        /* sum over completed requests */
    uint64_t hbm_used, hbm_budget;
    double elapsed_s;                          /* first arrival to last completion */
    uint64_t count[TP_SERVER_TAGS];            /* completed requests per tag */
    double p50_ms[TP_SERVER_TAGS];             /* arrival -> result latency per tag */
    double p99_ms[TP_SERVER_TAGS];
} tp_server_stats;

/* Create a server on the current device (synchronous).
 * Errors: TP_ERR_INVALID for out-of-range fields; TP_ERR_DEVICE. */
tp_status tripoll_server_create(const tp_server_config *cfg, tp_server **out);

/* Stop the worker and release every graph and buffer.  Requests not yet
 * complete are dropped.  NULL accepted. */
tp_status tripoll_server_destroy(tp_server *srv);

/*
 * Build a graph from `edges` (as tripoll_build) and keep it resident.  Its
 * bytes are taken from the budget: TP_ERR_OOM (and nothing kept) if they do
 * not fit.  Synchronous.  *graph_id receives its handle.
 */
tp_status tripoll_server_add_graph(tp_server *srv, const tp_edge_list *edges, uint32_t *graph_id);

/* Release a resident graph; TP_ERR_BUSY while requests on it wait or run,
 * TP_ERR_NOT_FOUND for an unknown id. */
tp_status tripoll_server_remove_graph(tp_server *srv, uint32_t graph_id);

/* Statistics of a resident graph. */
tp_status tripoll_server_graph_stats(tp_server *srv, uint32_t graph_id, tp_graph_stats *out);

/* The resident graph itself, borrowed (valid until it is removed), for
 * direct calls such as tripoll_survey; such calls may run beside the
 * server's own work. */
tp_status tripoll_server_graph(tp_server *srv, uint32_t graph_id, const tp_graph **out);

/*
 * Queue a survey of graph `graph_id`.  Returns at once with a ticket.
 * `tag` (0..7) groups requests for the latency statistics.
 * Errors: TP_ERR_NOT_FOUND (graph), TP_ERR_INVALID (spec as tripoll_survey;
 * labels used with n_labels other than the server's; DIRECTED on a graph
 * built without TP_EDGES_DIRECTED), TP_ERR_BUSY (queue full; the request is
 * not kept).
 */
tp_status tripoll_server_submit(tp_server *srv, uint32_t graph_id, const tp_survey_spec *spec, uint32_t tag,
                                uint64_t *ticket);

/*
 * Wait up to `timeout_us` (negative: no limit) for a request and take its
 * result: the counters of tripoll_survey (probes = the graph's wedge checks;
 * kernel_ms, class_ms 0; total_ms = admission to completion) and, if `info`
 * is not NULL, its timing.  A ticket can be taken once.
 * Errors: TP_ERR_BUSY when not complete in time (ticket kept),
 * TP_ERR_NOT_FOUND for an unknown or taken ticket, TP_ERR_DEVICE if the
 * device failed while it ran.
 */
tp_status tripoll_server_wait(tp_server *srv, uint64_t ticket, int64_t timeout_us, tp_survey_result *out,
                              tp_request_info *info);

/* Counters and latency percentiles (nearest rank over completed requests). */
tp_status tripoll_server_stats(tp_server *srv, tp_server_stats *out);

/* Colex index of the label multiset {a, b, c} (any order). */
uint32_t tripoll_msidx(uint32_t a, uint32_t b, uint32_t c);

/* Return the device memory cached by the library's allocator to the driver
 * (blocks kept after graphs and temporaries were released). */
tp_status tripoll_trim(void);

/* Bytes currently cached by the allocator on the current device. */
tp_status tripoll_cached_bytes(uint64_t *out);

/* Device bytes the library's allocator has handed out on the current device
 * and not yet released (graphs, servers, temporaries of calls in progress;
 * the cache of released blocks is not counted). */
tp_status tripoll_live_bytes(uint64_t *out);

/* Fault injection for tests of the error paths: the n-th device allocation
 * the library makes from now on (n >= 1, counted over all threads and
 * devices) fails once, as if the device were out of memory, so the call
 * making it returns TP_ERR_OOM and must release everything it took; n = 0
 * switches the injection off. */
tp_status tripoll_fail_alloc_after(uint64_t n);

/* Message of the last failed call on this thread ("" if none). */
const char *tripoll_last_error(void);

/* Library version string. */
const char *tripoll_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIPOLL_H */
