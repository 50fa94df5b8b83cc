// graph.hpp -- device layout of a built degree-ordered directed graph.
#pragma once

#include "tp_internal.hpp"

// One tile of survey work: `cnt` consecutive in-edge records of target q,
// starting at record e0.
struct TileDesc {
    uint32_t q;
    uint32_t cnt;
    uint64_t e0;
};

// In-edge record of target q for the oriented edge p -> q stored at CSR slot
// k of p's row: the wedges (p,q,r) to check are the rest of p's row after k.
//   w0 = k bits 0..31, w1 = k bits 32..55 | label(p) << 24,
//   w2 = length of the rest of p's row, w3 = time of edge (p,q).
struct InRec {
    uint32_t k_lo;
    uint32_t k_hi_lab;
    uint32_t len;
    uint32_t t_pq;
};

// Target classes of the survey plan, by d+(q).
enum { kClassSmall = 0, kClassLarge = 1, kClassHuge = 2, kNumClasses = 3 };

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
    tp::DArray<uint32_t> perm;    // [n] rank -> original id
    tp::DArray<InRec> inrec;      // [n_in] in-edge records grouped by target
    tp::DArray<TileDesc> tiles[kNumClasses];
    uint64_t n_tiles[kNumClasses] = {0, 0, 0};
    tp_graph_stats stats{};
};
