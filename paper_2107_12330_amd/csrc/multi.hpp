// multi.hpp -- multi-request passes over one resident graph (served mode).
//
// A pass runs the survey kernels once over a graph's tiles and reduces every
// triangle into the counters of several requests at once, each with its own
// outputs and prefilters (the callback of Algorithm 1 applied per request).
// A pass is cut into segments (equal shares of every target class's tiles);
// a request that joins at segment j has seen every tile once after it has
// taken part in segments j, j+1, ..., wrapping around, n_seg steps in all.
#pragma once

#include "graph.hpp"

namespace tp {

constexpr uint32_t kMaxSlots = 16;

// One request of a multi-request pass, in the form the kernel tests it.
// `off` set: the slot is unused and contributes nothing.
struct SlotSpec {
    uint32_t outputs, filters, t_lo, t_hi;
    uint32_t spread_le, spread_any, window_empty, off;
    uint64_t label_mask[13];
};

// Kernel form of a request.  Supported outputs: COUNT, CLOSE_HIST,
// LABEL_TABLE, SPREAD_COUNT; filters: WINDOW, LABEL_MASK.
SlotSpec make_slot(const tp_survey_spec &sp);

// Words of one slot's result block: the batch block layout (TP_BW_*), with
// the label table sized for `n_labels` labels.
uint32_t slot_words(uint32_t n_labels);

// Enqueue segment `seg` of `n_seg` of a pass over `g` on stream `s`:
// slots [0, n_slots) of `dev_slots` reduce into dev_out + slot * words.
// `dev_counter` is one device word of scratch.  `grid_eighths` in 1..8
// limits the persistent grid to that share of the device (8 = all of it),
// leaving compute units to work on other streams.  Allocates nothing.
void multi_segment_enqueue(const tp_graph *g, const SlotSpec *dev_slots, uint32_t n_slots, uint32_t n_labels,
                           bool labels, unsigned long long *dev_out, unsigned long long *dev_counter, uint32_t seg,
                           uint32_t n_seg, uint32_t grid_eighths, hipStream_t s);

// Enqueue segment `seg` of `n_seg` of a single-request pass: the survey of
// `sp` (any outputs and filters tripoll_survey takes, with the kernels it
// uses) over the same tiles as multi_segment_enqueue's segment, accumulated
// into a result block of TP_RESULT_WORDS words at `dev_out` (cleared by the
// caller before the first segment; its scratch words hold the tile counter).
// For served requests whose counters do not fit the shared pass.
void solo_segment_enqueue(const tp_graph *g, const tp_survey_spec *sp, unsigned long long *dev_out, uint32_t seg,
                          uint32_t n_seg, uint32_t grid_eighths, hipStream_t s);

// Zero `n` device words with a fill kernel (safe inside recorded graphs).
void zero_words(unsigned long long *p, size_t n, hipStream_t s);

}  // namespace tp
