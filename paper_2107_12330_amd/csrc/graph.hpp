// graph.hpp -- device layout of a built degree-ordered directed graph.
#pragma once

#include "tp_internal.hpp"

// One tile of survey work: `cnt` in-edge records of target q, records e0,
// e0 + stride, e0 + 2 stride, ...  (the tiles of a target interleave, so
// each gets a fair share of long and short rows), checked against piece
// `piece` of Adj+(q) (always 0 but for huge targets; see piece_count).
struct TileDesc {
    uint32_t q;
    uint32_t cnt;
    uint64_t e0;
    uint32_t stride;
    uint32_t piece;
};

// In-edge index: one entry per oriented edge p -> q whose remaining row is
// non-empty, sorted by q.  The key holds q above bit `kbits` and the CSR
// slot k of the edge in p's row below it; the wedges (p, q, r) to check are
// the slots after k in p's row.  A second array holds their number and
// label(p), so that the only gather of a record is the time of p -> q.
// Target classes of the survey plan, by d+(q).
enum { kClassTiny = 0, kClassSmall = 1, kClassLarge = 2, kClassHuge = 3, kNumClasses = TP_NUM_CLASSES };

// Survey plan choices per class: how Adj+(q) is searched (TP_VAR_*) and the
// records-per-tile cap the tiles were cut with.
struct PlanCfg {
    uint32_t variant[kNumClasses];
    uint32_t tile_records[kNumClasses];
};

struct tp_graph {
    int device = 0;
    uint32_t n = 0;       // vertices
    uint32_t nbits = 1;   // bits of a vertex id / rank
    uint64_t m = 0;       // unique undirected edges = oriented edges
    uint64_t n_in = 0;    // in-edge records
    tp::DArray<uint64_t> rowptr;  // [n+1] out-rows by rank
    tp::DArray<uint32_t> col;     // [m] target ranks, ascending in each row
    tp::DArray<uint32_t> ets;     // [m] edge times
    tp::DArray<uint8_t> tlab;     // [m] label of each target
    tp::DArray<uint8_t> rlab;     // [n] label by rank
    bool directed = false;        // built from a directed edge list
    tp::DArray<uint8_t> edir;     // [m + pad] directed builds: bit 0 arc source -> target, bit 1 the reverse
    tp::DArray<uint32_t> perm;    // [n] rank -> original id
    uint32_t kbits = 1;           // bits of a CSR slot in an in-edge key
    tp::DArray<uint64_t> inkey;   // [n_in] (q << kbits) | k, sorted by q
    tp::DArray<uint32_t> inpay;   // [n_in] rest of p's row after slot k | label(p) << 24
    // the in-edge records of huge targets cut to each piece of Adj+(q)
    // (plan.hpp): for every target and piece in turn, the records with
    // candidates in the piece, in in-edge order; key ((q + skip) << kbits) | k
    // with skip the candidates below the piece's ranks, payload the
    // candidates in the piece | label(p) << 24
    uint64_t n_piece_recs = 0;
    tp::DArray<uint64_t> piece_key;
    tp::DArray<uint32_t> piece_pay;
    tp::DArray<TileDesc> tiles[kNumClasses];
    // degree bins (bin(d) = ceil(log2 d), 0 for d <= 1): ranks are in degree
    // order, so each bin is a range of ranks and of CSR slots (single graphs)
    uint32_t dbin_values = 0;          // bin(d_max) + 1
    tp::DArray<uint32_t> dbin_rank;    // [32 per graph] first rank of bin >= k, or 2^32 - 1
    tp::DArray<uint64_t> dbin_slot;    // [32 per graph] first CSR slot of a rank of bin >= k, or 2^64 - 1
    uint32_t n_graphs = 0;         // > 0 for a batch of disjoint graphs
    tp::DArray<uint32_t> rank_gid; // [n] graph of each rank (batches only)
    uint64_t n_tiles[kNumClasses] = {};
    PlanCfg plan{};
    tp_graph_stats stats{};
};

// Cut the survey tiles of every class with the caps of `cfg`, store `cfg` as
// the graph's plan and refresh the plan statistics (build.hip).
void plan_graph(tp_graph *g, const PlanCfg &cfg, hipStream_t s);

// Device bytes held by a graph.
uint64_t graph_bytes(const tp_graph *g);
