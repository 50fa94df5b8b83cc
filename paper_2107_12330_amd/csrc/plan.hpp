// plan.hpp -- sizes shared by the survey planner (build) and the survey
// kernels.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace tp {

// Targets q are split into classes by d+(q): the class decides how Adj+(q)
// is searched.  Tiny, small and large targets keep a two-table cuckoo hash
// of Adj+(q) in LDS (each table 2^k >= 1.25 d+(q) slots, so the load stays
// at most 0.4, plus a small stash); tiny ones get one table per wave, small
// and large ones one per workgroup.  Huge targets are surveyed in pieces of
// Adj+(q) that fit the large class's tables (below).
constexpr uint32_t kTinyMaxDeg = 51;     // per-wave tables of <= 64 slots
constexpr uint32_t kSmallMaxDeg = 819;   // tables of <= 1024 slots
constexpr uint32_t kLargeMaxDeg = 3276;  // tables of <= 4096 slots
constexpr int kTinyLogSlots = 6;
constexpr int kSmallLogSlots = 10;
constexpr int kLargeLogSlots = 12;
constexpr uint32_t kStash = 32;          // keys the cuckoo insertion could not place

// Pieces of a huge target.  Adj+(q) is sorted by rank; it is cut into
// S = ceil(d+(q) / kLargeMaxDeg) runs of P = ceil(d+(q) / S) slots (the last
// one shorter), piece j holding slots [jP, min((j + 1)P, d+(q))).  Piece j
// owns the ranks from its first key up to the first key of piece j + 1 (the
// first piece from 0, the last one to the top), so these ranges partition
// the ranks and every candidate r of an in-edge record is checked against
// exactly one piece: the one whose range holds r.  Targets with
// d+(q) <= kLargeMaxDeg are one piece.
__host__ __device__ inline uint32_t piece_count(uint64_t dq)
{
    return dq > kLargeMaxDeg ? (uint32_t)((dq + kLargeMaxDeg - 1) / kLargeMaxDeg) : 1u;
}
__host__ __device__ inline uint32_t piece_size(uint64_t dq)
{
    const uint64_t s = piece_count(dq);
    return (uint32_t)((dq + s - 1) / s);
}

// A tile holds at most `cap` in-edge records of one target (of one piece of
// a huge target) and about kTileWorkPerRecord * cap wedge checks.  Default
// caps: 1024 records, and 16384 for the large and huge classes, whose
// workgroups stall for the first records of every tile; the tuner may choose
// others.
constexpr uint32_t kTileRecords = 1024;
constexpr uint64_t kTileWorkPerRecord = 256;
inline uint32_t default_tile_records(int cls) { return cls >= 2 ? 16384u : kTileRecords; }

// Slots of padding after the last oriented edge in the target and time
// arrays, so that a wave may load 64 consecutive slots from any row start.
constexpr uint64_t kRowPad = 64;

}  // namespace tp
